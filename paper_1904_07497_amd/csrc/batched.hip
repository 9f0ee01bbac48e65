// Batched RES-PCA: many independent instances of uneven d, n and c solved by one
// persistent kernel launch (replayed from a hipGraph).
//
// Every instance runs its own copy of the method -- initial K-means, then outer
// ALM iterations (Sec. 4.1 -> 4.2 -> 4.3 -> 4.4) with its own iteration count,
// Lloyd passes and Sec. 5 stopping test -- as a small state machine.  The grid
// walks a fixed sequence of phases; in each phase the work items (instance,
// tile) of all instances whose state needs that phase are spread over every
// workgroup, and phases are separated by a grid barrier.  The barrier's wait is
// bounded by a wall-clock limit: a workgroup that waits too long raises an abort
// flag that every other wait sees, so the launch always drains and the host
// reports an error instead of hanging.
//
// An instance given an embedding (a few rows per column, e.g. a learned warm
// start's predicted sketches) runs its initial K-means on the embedding's
// columns instead of X's, then takes the means of X over the resulting groups
// (empty groups at zero) and starts the iterations from there.
//
// Instances are stored zero-padded to d' = 4 * ceil(d / 4) rows so every tile
// takes the 16-byte vector path; the padding rows stay exactly zero through all
// steps (X, S, Theta, centroids and hence L are zero there), so sums, norms and
// dot products are those of the unpadded problem.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "batched.h"
#include "device_common.h"
#include "dist_tile.h"

static_assert(respca::kBatchSegCols <= respca::kMaxSegCols, "segments must fit the LDS column list");

namespace respca {

namespace {

// M_SEED / M_KMX: k-means++ and Lloyd on X, or on the embedding when given one;
// M_MEANSX: centroids = means of X over given groups (empty groups at zero);
// M_REFX: Lloyd on X from the embedding's groups; M_ITER: an outer iteration with
// its first Lloyd pass on L; M_LL: further Lloyd passes on L.
enum Mode : int { M_DONE = 0, M_SEED = 1, M_MEANSX = 2, M_KMX = 3, M_ITER = 4, M_LL = 5, M_REFX = 6 };

// ---------------------------------------------------------------- barrier

// Two-level grid barrier.  Workgroups arrive on one of eight group counters
// (workgroup index mod 8, each on its own cache line), the last arrival of each
// group on the top counter, and the last top arrival bumps the generation the
// others poll.  Memory ordering uses fences instead of ordered atomics: one
// agent-scope release fence before arriving, an acquire-release fence in every
// last arrival (which passes the earlier arrivals' writes on), relaxed polling
// and one acquire fence after it -- so each wait costs one cache write-back and
// one invalidate instead of one per poll.  Every wait is bounded by a wall-clock
// limit; a workgroup that waits too long raises the abort flag, which ends every
// other wait, and all workgroups then leave the kernel.
__device__ bool grid_sync(BatchSync* gs, unsigned nblocks, uint64_t timeout_ticks, int phase,
                          uint64_t& t_prev) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            const unsigned g = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned grp = blockIdx.x & 7u;
            unsigned* gc = &gs->group_count[grp * 64];
            const unsigned members = (nblocks - grp + 7u) / 8u;
            bool waiter = true;
            if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
                __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                const unsigned groups = nblocks < 8u ? nblocks : 8u;
                if (__hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                    groups - 1) {
                    __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                    __hip_atomic_fetch_add(&gs->gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    waiter = false;
                }
            }
            if (waiter) {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                    if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                    if (wall_clock64() - t0 > timeout_ticks) {
                        __hip_atomic_store(&gs->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        s_ok = __hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 0 : 1;
        if (blockIdx.x == 0) {   // phase time as seen by one workgroup: its work plus the wait
            const uint64_t t = wall_clock64();
            gs->phase_ticks[phase] += t - t_prev;
            t_prev = t;
        }
    }
    __syncthreads();
    return s_ok != 0;
}

// ------------------------------------------------------------ item lookup

// Largest i with off[i] <= item (off is a prefix table of batch + 1 entries).
__device__ inline int find_inst(const int32_t* __restrict__ off, int batch, int item) {
    int lo = 0, hi = batch;   // off[lo] <= item < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ inline bool needs_groups(int m) {
    return m == M_MEANSX || m == M_KMX || m == M_ITER || m == M_LL || m == M_REFX;
}
__device__ inline bool needs_assign(int m) {
    return m == M_SEED || m == M_KMX || m == M_ITER || m == M_LL || m == M_REFX;
}

// Modes whose means pass is a Lloyd step on an unchanged matrix (the sums can be
// carried from one step to the next).
__device__ inline bool lloyd_family(int m) { return m == M_KMX || m == M_LL || m == M_REFX; }

// Segments of the moved-column sort for `moved` columns (2 entries each, at most
// 2c keys), as in changed_max_segments.
__device__ inline int moved_segments(int moved, int c) {
    const int e = 2 * moved;
    return (e + kBatchSegCols - 1) / kBatchSegCols + min(2 * c, e);
}

// Matrix whose columns the current mode clusters, and its row count (= its
// leading dimension and that of the centroids).
// (With seed_only the embedding serves the seeding distances alone: the nearest-
// seed assignment and the K-means that follows run on X.)
__device__ inline bool kmeans_on_z(const BatchInst& B) { return B.Z && !B.seed_only; }
__device__ inline const float* kmeans_matrix(const BatchInst& B, int m) {
    if (m == M_ITER || m == M_LL) return B.L;
    if (m == M_MEANSX || m == M_REFX) return B.X;
    return kmeans_on_z(B) ? B.Z : B.X;
}
__device__ inline int mode_rows(const BatchInst& B, int m) {
    return (m == M_SEED || m == M_KMX) && kmeans_on_z(B) ? B.kdp : B.dp;
}

// ------------------------------------------------------- per-instance work

// Stable counting sort of one instance's labels by one workgroup, with the
// segment table of the means pass (runs of <= kBatchSegCols columns of one group).
// With old labels (2c <= kMaxGroups) it sorts only the moved columns instead:
// column j with old[j] = a != lab[j] = b is listed under key b (entering) and key
// c + a (leaving), keys in order and columns in order within a key; the segment
// table then has 2c + 1 entries in segf and the counts become those of lab.
__device__ void sort_instance(BatchInst& B, const int32_t* __restrict__ lab,
                              const int32_t* __restrict__ old = nullptr) {
    __shared__ int hist[kMaxGroups];
    __shared__ int offs[kMaxGroups];
    __shared__ int wsum[kBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = B.n, c = B.c;
    const int K = old ? 2 * c : c;   // keys
    for (int k = tid; k < K; k += kBlock) hist[k] = 0;
    __syncthreads();
    if (old) {
        for (int j = tid; j < n; j += kBlock) {
            const int a = old[j], b = lab[j];
            if (a != b) {
                atomicAdd(&hist[b], 1);
                atomicAdd(&hist[c + a], 1);
            }
        }
    } else {
        for (int j = tid; j < n; j += kBlock) atomicAdd(&hist[lab[j]], 1);
    }
    __syncthreads();
    // each thread owns 4 consecutive groups; two block exclusive scans
    int cnt[4], nsg[4], my_c = 0, my_s = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int k = tid * 4 + g;
        cnt[g] = k < K ? hist[k] : 0;
        nsg[g] = (cnt[g] + kBatchSegCols - 1) / kBatchSegCols;
        my_c += cnt[g];
        my_s += nsg[g];
    }
    auto exscan = [&](int v) -> int {
        int x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        __syncthreads();
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int base = 0;
        for (int w = 0; w < wave; ++w) base += wsum[w];
        return base + x - v;
    };
    int bc = exscan(my_c);
    int bs = exscan(my_s);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int k = tid * 4 + g;
        if (k < K) {
            offs[k] = bc;
            if (!old) B.counts[k] = cnt[g];
            B.segf[k] = bs;
            for (int q = 0; q < nsg[g]; ++q) {
                B.segb[bs + q] = bc + q * kBatchSegCols;
                B.segl[bs + q] = min(kBatchSegCols, cnt[g] - q * kBatchSegCols);
            }
            if (k == K - 1) { B.segf[K] = bs + nsg[g]; B.nseg = bs + nsg[g]; }
        }
        bc += cnt[g];
        bs += nsg[g];
    }
    if (old)   // counts of the new labels: entering minus leaving
        for (int k = tid; k < c; k += kBlock) B.counts[k] += hist[k] - hist[c + k];
    __syncthreads();
    // stable scatter by wave 0, 64 columns at a time: the lanes holding the same
    // label are found with one ballot per label bit; a lane's rank among them is
    // the count of such lanes below it, and the lowest of them advances the offset.
    if (wave == 0) {
        int nbits = 0;
        while ((1 << nbits) < K) ++nbits;
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        // pass 0: every column under its label, or (old) the entering keys; pass 1
        // (old only): the leaving keys
        // the labels of the next PF chunks are loaded while a chunk is placed
        // (loads clamped into the columns, no branch around them)
        constexpr int PF = 4;
        const int nch = (n + 63) / 64;
        int la[PF], lo[PF];
        auto fetch = [&](int ch, int slot) {
            const int jj = min(min(ch, nch - 1) * 64 + lane, n - 1);
            la[slot] = lab[jj];
            lo[slot] = old ? old[jj] : 0;
        };
        for (int pass = 0; pass < (old ? 2 : 1); ++pass) {
#pragma unroll
            for (int q = 0; q < PF; ++q) fetch(q, q);
            for (int ch0 = 0; ch0 < nch; ch0 += PF)
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                if (ch0 + q >= nch) break;
                const int j = (ch0 + q) * 64 + lane;
                const int lb = la[q], lold = lo[q];
                fetch(ch0 + q + PF, q);
                bool valid = j < n;
                int my = 0;
                if (valid) {
                    if (!old) {
                        my = lb;
                    } else {
                        valid = lold != lb;
                        my = pass == 0 ? lb : c + lold;
                    }
                }
                uint64_t same = __ballot(valid);
                if (same == 0) continue;   // nothing of this pass in these 64 columns
                for (int b = 0; b < nbits; ++b) {
                    const bool bit = (my >> b) & 1;
                    const uint64_t m = __ballot(bit);
                    same &= bit ? m : ~m;
                }
                const int rank = __popcll(same & below);
                const int base_off = offs[my];
                if (valid) {
                    B.perm[base_off + rank] = j;
                    if (rank == 0) offs[my] = base_off + __popcll(same);
                }
            }
        }
    }
    __syncthreads();   // the tables are reused by the next instance of this workgroup
}

// k-means++ draw of seed m (m >= 1) for one instance by one workgroup; see k_pick.
__device__ void pick_instance(BatchInst& B, int m) {
    __shared__ double wtot[kBlock / 64];
    __shared__ int ish[kBlock / 64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int n = B.n;
    const int chunk = (n + kBlock - 1) / kBlock;
    const int lo = tid * chunk, hi = min(n, lo + chunk);
    double loc = 0.0;
    for (int j = lo; j < hi; ++j) loc += B.d2[j];
    double x = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    double pre = 0.0, total = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) pre += wtot[w];
        total += wtot[w];
    }
    pre += x - loc;
    auto bmin = [&](int v) -> int {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
        __syncthreads();
        if (lane == 0) ish[wave] = v;
        __syncthreads();
        int r = ish[0];
        for (int w = 1; w < kBlock / 64; ++w) r = min(r, ish[w]);
        return r;
    };
    int s;
    if (total > 0.0) {
        const double target = B.u[m] * total;
        int cand = INT_MAX;
        double run = pre;
        for (int j = lo; j < hi; ++j) {
            run += B.d2[j];
            if (run > target) { cand = j; break; }
        }
        s = bmin(cand);
        if (s == INT_MAX) {
            int last = INT_MAX;
            for (int j = hi - 1; j >= lo; --j)
                if (B.d2[j] > 0.0) { last = -j; break; }
            s = -bmin(last);
        }
    } else {
        int cand = INT_MAX;
        for (int j = lo; j < hi; ++j)
            if (!B.chosen[j]) { cand = j; break; }
        s = bmin(cand);
    }
    if (tid == 0) { B.seeds[m] = s; B.chosen[s] = 1; }
}

// Control step of one instance: the workgroup sums the changed counts and (for
// an outer iteration) the sweep's norm partials in fixed order, then thread 0
// updates the state.
__device__ void control_instance(BatchInst& B, int* active) {
    __shared__ int s_mode;
    if (threadIdx.x == 0) s_mode = B.mode;
    __syncthreads();
    const int mode0 = s_mode;
    if (!needs_assign(mode0) && mode0 != M_MEANSX) return;
    double ch = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0, z = 0.0;
    if (mode0 != M_MEANSX) {
        for (int t = threadIdx.x; t < 4 * B.n_argmin; t += kBlock) ch += (double)B.chg[t];
        if (mode0 == M_ITER)
            for (int t = threadIdx.x; t < B.n_sweep; t += kBlock) {
                a0 += B.sweep_part[3 * t];
                a1 += B.sweep_part[3 * t + 1];
                a2 += B.sweep_part[3 * t + 2];
            }
    }
    block_sum3(ch, z, z);
    block_sum3(a0, a1, a2);
    if (threadIdx.x != 0) return;
    const int mode = mode0;
    B.pmode = mode;
    if (mode == M_MEANSX) {   // embedding groups: Lloyd on X next, once; then the iterations
        if (B.Z && B.refine_x && B.ref_lloyd == 0) { B.mode = M_REFX; } else { B.mode = M_ITER; }
        return;
    }
    const int changed = (int)ch;
    B.moved = changed;
    if (mode == M_SEED) { B.cur ^= 1; B.mode = M_KMX; return; }
    if (mode == M_KMX) {
        B.init_lloyd += 1;
        if (changed == 0 || B.init_lloyd >= B.max_lloyd) {
            if (changed) B.cur ^= 1;
            B.mode = kmeans_on_z(B) ? M_MEANSX : M_ITER;   // embedding groups: means of X next
        } else {
            B.cur ^= 1;
        }
        return;
    }
    if (mode == M_REFX) {
        B.init_lloyd += 1;
        B.ref_lloyd += 1;
        if (changed) B.cur ^= 1;
        if (changed == 0 || B.ref_lloyd >= B.max_lloyd) B.mode = M_MEANSX;   // means over the final groups
        return;
    }
    if (mode == M_ITER) {
        if (!B.next_ready) B.meansd += 1;   // this step's L-step summed D in the means phase
        B.iters += 1;
        B.rho_final = B.rho;
        B.primal = sqrt(a0) / B.nx;
        B.dL = sqrt(a1) / B.nx;
        B.dS = sqrt(a2) / B.nx;
        B.lloyd_iter = 0;
    }
    B.lloyd_iter += 1;
    B.lloyd_total += 1;
    // an outer iteration whose first assignment kept every label leaves the next
    // L-step's group sums (summed by this step's sweep) and the sort tables valid
    B.next_ready = (mode == M_ITER && changed == 0) ? 1 : 0;
    if (changed != 0 && B.lloyd_iter < B.max_lloyd) {
        B.cur ^= 1;
        B.mode = M_LL;
        return;
    }
    if (changed) B.cur ^= 1;
    B.rho_prev = B.rho;   // the penalty this iteration's sweep used
    const double next = B.kappa * B.rho;
    B.rho = next < B.rho_max ? next : B.rho_max;
    const double crit = fmax(B.primal, fmax(B.dL, B.dS));
    if (crit <= B.tol) {
        B.status = 0;
        B.mode = M_DONE;
        atomicSub(active, 1);
    } else if (B.iters >= B.max_iter) {
        B.status = 1;
        B.mode = M_DONE;
        atomicSub(active, 1);
    } else {
        B.mode = M_ITER;
    }
}

// --------------------------------------------------------------- kernel

// Work-item walk of one phase: items item = blockIdx.x + k * gridDim.x of the
// prefix table `tab` (cached in LDS), instance found by a forward scan; an
// instance that does not need the phase (need(mode, instance) false) is skipped
// in one step.
template <typename Need, typename Body>
__device__ inline void for_items(int batch, const int* tab, const int* modes, Need need, Body body) {
    const unsigned nb = gridDim.x;
    const int total = tab[batch];
    int i = 0;
    int item = blockIdx.x;
    while (item < total) {
        while (tab[i + 1] <= item) ++i;
        if (!need(modes[i], i)) {
            const int next = tab[i + 1];
            item = next + (int)((blockIdx.x + nb - (unsigned)next % nb) % nb);
            continue;
        }
        body(i, item - tab[i]);
        item += nb;
    }
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_batched(BatchArgs A) {
    BatchInst* __restrict__ inst = A.inst;
    const int batch = A.batch;
    const unsigned nb = gridDim.x;
    const uint64_t tmo = A.timeout_ticks;
    BatchSync* gs = A.sync;
    int* active = &A.sync->active;
    uint64_t tclk = wall_clock64();
    __shared__ int s_tab[kMaxBatch + 1];
    __shared__ int s_mode[kMaxBatch];
    __shared__ int s_nseg[kMaxBatch];
    __shared__ int s_ready[kMaxBatch];   // the instance skips its sort and means this step
    auto load_tab = [&](const int32_t* off) {
        __syncthreads();
        for (int t = threadIdx.x; t <= batch; t += kBlock) s_tab[t] = off[t];
        __syncthreads();
    };
    auto load_modes = [&]() {
        __syncthreads();
        for (int t = threadIdx.x; t < batch; t += kBlock) {
            const int m = __hip_atomic_load(&inst[t].mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_mode[t] = m;
            s_ready[t] = m == M_ITER && __hip_atomic_load(&inst[t].next_ready, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    };
    auto any = [](int, int) { return true; };
    auto groups = [](int m, int) { return needs_groups(m); };
    auto assigns = [](int m, int) { return needs_assign(m); };

    // ---- phase: copy X into its zero-padded internal copy; zero L, S, Theta;
    //      sums of squares of X
    load_tab(A.off_tile);
    for (int t = threadIdx.x; t < batch; t += kBlock) s_mode[t] = 1;
    __syncthreads();
    for_items(batch, s_tab, s_mode, any, [&](int i, int local) {
        BatchInst& B = inst[i];
        const int cb = local / B.nrb, rb = local % B.nrb;
        const int64_t j0 = (int64_t)cb * B.jc, j1 = min((int64_t)B.n, j0 + B.jc);
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;   // wave per column, 4 rows per lane
        const int64_t r = (int64_t)rb * kBatchRows + lane * 4;
        double a = 0.0, b = 0.0, c = 0.0;
        if (r < B.dp) {
            // up to four of the wave's columns at a time: every load (clamped into the
            // matrix, values past row d zeroed after) issued before the stores, the
            // columns' squares added in column order
            constexpr int PJ = 4, WS = kBlock / 64;
            for (int64_t jb = j0 + w; jb < j1; jb += PJ * WS) {
                float v[PJ][4];
#pragma unroll
                for (int u = 0; u < PJ; ++u) {
                    const int64_t j = jb + u * WS < j1 ? jb + u * WS : j1 - 1;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float t = B.Xc[j * B.ldx + (r + e < B.d ? r + e : B.d - 1)];
                        v[u][e] = r + e < B.d ? t : 0.f;
                    }
                }
#pragma unroll
                for (int u = 0; u < PJ; ++u) {
                    const int64_t j = jb + u * WS;
                    if (j >= j1) break;
                    const float4 x = make_float4(v[u][0], v[u][1], v[u][2], v[u][3]);
                    *reinterpret_cast<float4*>(B.X + j * B.dp + r) = x;
                    a += (double)x.x * x.x + (double)x.y * x.y + (double)x.z * x.z + (double)x.w * x.w;
                    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                    *reinterpret_cast<float4*>(B.L + j * B.dp + r) = z;
                    *reinterpret_cast<float4*>(B.S + j * B.dp + r) = z;   // B = 0: S = Theta = 0
                }
            }
        }
        if (B.Z && rb == 0)
            for (int64_t j = j0 + w; j < j1; j += kBlock / 64)
                for (int64_t q = lane * 4; q < B.kdp; q += 256) {
                    float v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (q + e < B.er) ? B.Ec[j * B.lde + q + e] : 0.f;
                    *reinterpret_cast<float4*>(B.Z + j * B.kdp + q) = make_float4(v[0], v[1], v[2], v[3]);
                }
        block_sum3(a, b, c);
        if (threadIdx.x == 0) B.sweep_part[3 * local] = a;
    });
    if (!grid_sync(gs, nb, tmo, BP_PACK, tclk)) return;

    // ---- phase: initial state of every instance
    for (int i = blockIdx.x; i < batch; i += nb) {
        BatchInst& B = inst[i];
        __shared__ int s_m, s_status;
        double nx2 = 0.0, z1 = 0.0, z2 = 0.0;
        for (int t = threadIdx.x; t < B.n_tile; t += kBlock) nx2 += B.sweep_part[3 * t];
        block_sum3(nx2, z1, z2);
        if (threadIdx.x == 0) {
            B.nx = sqrt(nx2);
            B.cur = 0;
            B.iters = B.lloyd_total = B.lloyd_iter = B.init_lloyd = B.ref_lloyd = 0;
            B.next_ready = 0;
            B.meansd = 0;
            B.pmode = M_DONE;
            B.moved = 0;
            B.inc = 0;
            B.inc_steps[0] = B.inc_steps[1] = 0;
            B.inc_cols[0] = B.inc_cols[1] = 0;
            B.rho = B.rho0;
            B.rho_prev = B.rho0;   // B = 0 stands for S = Theta = 0 at any penalty
            B.rho_final = 0.0;
            B.primal = B.dL = B.dS = 0.0;
            B.nseg = 0;
            if (!isfinite(nx2)) { B.status = -2; B.mode = M_DONE; atomicSub(active, 1); }
            else if (nx2 == 0.0) { B.status = 0; B.mode = M_DONE; atomicSub(active, 1); }
            else { B.status = 1; B.mode = B.init_labels ? M_MEANSX : M_SEED; }
            s_m = B.mode;
            s_status = B.status;
        }
        __syncthreads();
        const int m = s_m;
        if (s_status == 0 && m == M_DONE)
            for (int j = threadIdx.x; j < B.n; j += kBlock) B.lab[0][j] = 0;
        if (m == M_MEANSX)
            for (int j = threadIdx.x; j < B.n; j += kBlock) B.lab[0][j] = B.init_labels[j];
        if (m == M_SEED) {
            for (int j = threadIdx.x; j < B.n; j += kBlock) B.chosen[j] = 0;
            __syncthreads();
            if (threadIdx.x == 0) {
                int64_t s0 = (int64_t)floor(B.u[0] * (double)B.n);
                if (s0 >= B.n) s0 = B.n - 1;
                B.seeds[0] = (int)s0;
                B.chosen[s0] = 1;
            }
        }
        __syncthreads();
    }
    if (!grid_sync(gs, nb, tmo, BP_INIT, tclk)) return;
    load_modes();

    // ---- k-means++ seeding, seed by seed, for instances in M_SEED
    auto is_seed = [](int m, int) { return m == M_SEED; };
    for (int m = 0; m < A.cmax; ++m) {
        load_tab(A.off_d2);
        // instances with fewer seeds than m + 1 are skipped whole
        auto seeds_m = [&](int mode, int i) { return mode == M_SEED && m < inst[i].c; };
        for_items(batch, s_tab, s_mode, seeds_m, [&](int i, int local) {
            BatchInst& B = inst[i];
            const int lane = threadIdx.x & 63;
            const float* Y = B.Z ? B.Z : B.X;
            const int rows = B.kdp;
            const float* ys = Y + (int64_t)B.seeds[m] * rows;
            // 16 columns per item, four per wave together: each 512-row pass loads
            // the seed rows once and the four columns' rows beside them (rows is a
            // multiple of 4, zero padded; columns past n read column n - 1)
            constexpr int NC4 = 4;
            int64_t j[NC4];
            const float* yj[NC4];
#pragma unroll
            for (int t = 0; t < NC4; ++t) {
                j[t] = (int64_t)local * 16 + (threadIdx.x >> 6) * NC4 + t;
                yj[t] = Y + (j[t] < B.n ? j[t] : B.n - 1) * rows;
            }
            double acc[NC4];
            d2_columns<NC4>(yj, ys, rows, lane, acc);
#pragma unroll
            for (int t = 0; t < NC4; ++t)
                if (lane == 0 && j[t] < B.n) B.d2[j[t]] = (m == 0) ? acc[t] : fmin(B.d2[j[t]], acc[t]);
        });
        if (!grid_sync(gs, nb, tmo, BP_SEED_D2, tclk)) return;
        if (m + 1 >= A.cmax) break;
        for (int i = blockIdx.x; i < batch; i += nb) {
            BatchInst& B = inst[i];
            if (s_mode[i] == M_SEED && m + 1 < B.c) pick_instance(B, m + 1);
        }
        if (!grid_sync(gs, nb, tmo, BP_SEED_PICK, tclk)) return;
    }
    // centroids = seed columns
    load_tab(A.off_kc);
    for_items(batch, s_tab, s_mode, is_seed, [&](int i, int k) {
        BatchInst& B = inst[i];
        const int rows = mode_rows(B, M_SEED);
        const float* src = kmeans_matrix(B, M_SEED) + (int64_t)B.seeds[k] * rows;
        for (int64_t r = threadIdx.x; r < rows; r += kBlock) B.C[(int64_t)k * rows + r] = src[r];
    });
    if (!grid_sync(gs, nb, tmo, BP_GATHER, tclk)) return;

    // ---- main loop: one step of every live instance per pass
    for (int step = 0; step < A.max_steps; ++step) {
        if (__hip_atomic_load(active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0) break;
        load_modes();
        // A: sort the current labels
        for (int i = blockIdx.x; i < batch; i += nb) {
            BatchInst& B = inst[i];
            const int m = s_mode[i];
            // a Lloyd-family step after one of the same mode that moved few columns
            // updates the previous step's sums from the moved columns only
            const bool inc = needs_groups(m) && !s_ready[i] && lloyd_family(m) && B.pmode == m &&
                             2 * B.c <= kMaxGroups && B.moved <= B.n / 8 &&
                             moved_segments(B.moved, B.c) <= (B.n + kBatchSegCols - 1) / kBatchSegCols + B.c;
            if (needs_groups(m) && !s_ready[i])
                sort_instance(B, B.lab[B.cur], inc ? B.lab[B.cur ^ 1] : nullptr);
            if (threadIdx.x == 0) {
                B.inc = inc ? 1 : 0;
                if (inc) {
                    const int z = (m == M_KMX && kmeans_on_z(B)) ? 1 : 0;
                    B.inc_steps[z] += 1;
                    B.inc_cols[z] += 2 * (int64_t)B.moved;
                }
            }
        }
        if (!grid_sync(gs, nb, tmo, BP_SORT, tclk)) return;
        for (int t = threadIdx.x; t < batch; t += kBlock)
            s_nseg[t] = needs_groups(s_mode[t]) ? __hip_atomic_load(&inst[t].nseg, __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_AGENT) : 0;
        // B: group partial sums (of X, of D = X - S + Theta/rho, or of L)
        load_tab(A.off_seg);
        for_items(batch, s_tab, s_mode, [&](int m, int i) { return needs_groups(m) && !s_ready[i]; }, [&](int i, int local) {
            BatchInst& B = inst[i];
            const int mode = s_mode[i];
            const int s = local / B.mrb, rb = local % B.mrb;
            if (s >= s_nseg[i]) return;
            const int rows = mode_rows(B, mode);
            const int64_t r0 = (int64_t)rb * kBatchRows;
            if (r0 >= rows) return;
            double* out = B.pmeans + (int64_t)s * rows;
            if (mode == M_ITER)   // D from the compact state B of the last sweep
                group_partial_tile<float, 4, true, kBatchRows, 4, true>(
                    B.X, B.dp, B.S, B.dp, nullptr, 0, (float)(1.0 / B.rho), B.dp, B.perm, B.segb[s],
                    B.segl[s], r0, out, (float)B.rho_prev, (float)(1.0 / B.rho_prev));
            else
                group_partial_tile<float, 4, false, kBatchRows, 4>(
                    kmeans_matrix(B, mode), rows, nullptr, 0, nullptr, 0, 0.f, rows, B.perm,
                    B.segb[s], B.segl[s], r0, out);
        });
        if (!grid_sync(gs, nb, tmo, BP_MEANS, tclk)) return;
        // C: centroids (group means; an empty group keeps its centroid, except the
        //    means of X over given groups, where it is zero) and their squared norms,
        //    one workgroup per (instance, group)
        load_tab(A.off_kc);
        for_items(batch, s_tab, s_mode, [](int m, int) { return needs_groups(m) || needs_assign(m); },
                  [&](int i, int k) {
            BatchInst& B = inst[i];
            const int mode = s_mode[i];
            const int rows = mode_rows(B, mode);
            float* Ck = B.C + (int64_t)k * rows;
            double* Gk = B.gsum + (int64_t)k * rows;
            double a = 0.0, zb = 0.0, zc = 0.0;
            if (needs_groups(mode) && B.inc) {
                // incremental: sums plus entering minus leaving partials, in segment order
                const int e0 = B.segf[k], e1 = B.segf[k + 1];
                const int l0 = B.segf[B.c + k], l1 = B.segf[B.c + k + 1];
                if (e0 == e1 && l0 == l1) return;   // no column entered or left: C and its norm stay
                const int nk = B.counts[k];
                // four rows per thread at a time (loads clamped into the rows); each
                // row's partials added in segment order, the squares in row order
                constexpr int RU = 4;
                for (int64_t r0 = threadIdx.x; r0 < rows; r0 += RU * kBlock) {
                    float cv[RU];
                    double gk[RU], add[RU], sub[RU];
#pragma unroll
                    for (int q = 0; q < RU; ++q) {
                        const int64_t r = r0 + q * kBlock < rows ? r0 + q * kBlock : rows - 1;
                        cv[q] = Ck[r];
                        gk[q] = Gk[r];
                        add[q] = 0.0;
                        sub[q] = 0.0;
                    }
                    if (nk != 0) {
                        for (int g = e0; g < e1; ++g) {
                            double t[RU];
#pragma unroll
                            for (int q = 0; q < RU; ++q)
                                t[q] = B.pmeans[(int64_t)g * rows +
                                                (r0 + q * kBlock < rows ? r0 + q * kBlock : rows - 1)];
#pragma unroll
                            for (int q = 0; q < RU; ++q) add[q] += t[q];
                        }
                        for (int g = l0; g < l1; ++g) {
                            double t[RU];
#pragma unroll
                            for (int q = 0; q < RU; ++q)
                                t[q] = B.pmeans[(int64_t)g * rows +
                                                (r0 + q * kBlock < rows ? r0 + q * kBlock : rows - 1)];
#pragma unroll
                            for (int q = 0; q < RU; ++q) sub[q] += t[q];
                        }
                    }
#pragma unroll
                    for (int q = 0; q < RU; ++q) {
                        const int64_t r = r0 + q * kBlock;
                        if (r >= rows) break;
                        float v = cv[q];
                        if (nk == 0) {
                            Gk[r] = 0.0;   // emptied: the centroid stays, its sum is exactly zero
                        } else {
                            const double sum = gk[q] + (add[q] - sub[q]);
                            Gk[r] = sum;
                            v = (float)(sum / (double)nk);
                            Ck[r] = v;
                        }
                        a += (double)v * (double)v;
                    }
                }
            } else if (needs_groups(mode)) {
                const int nk = B.counts[k];
                const int g0 = B.segf[k], g1 = B.segf[k + 1];
                const bool keep = lloyd_family(mode);   // sums carried to the next Lloyd step
                if (nk == 0) {
                    for (int64_t r = threadIdx.x; r < rows; r += kBlock) {
                        const float v = mode == M_MEANSX ? 0.f : Ck[r];
                        if (mode == M_MEANSX) Ck[r] = 0.f;
                        if (keep) Gk[r] = 0.0;
                        a += (double)v * (double)v;
                    }
                } else {
                    // four rows per thread at a time, each with four segments' loads in
                    // flight (clamped: no branch per load); every row's segments are
                    // added in order and the rows' squares in row order
                    constexpr int RU = 4;
                    for (int64_t r0 = threadIdx.x; r0 < rows; r0 += RU * kBlock) {
                        double sum[RU];
#pragma unroll
                        for (int q = 0; q < RU; ++q) sum[q] = 0.0;
                        for (int g = g0; g < g1; g += 4) {
                            double v[RU][4];
#pragma unroll
                            for (int q = 0; q < RU; ++q) {
                                const int64_t r = r0 + q * kBlock < rows ? r0 + q * kBlock : rows - 1;
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    v[q][u] = B.pmeans[(int64_t)(g + u < g1 ? g + u : g1 - 1) * rows + r];
                            }
#pragma unroll
                            for (int q = 0; q < RU; ++q)
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    if (g + u < g1) sum[q] += v[q][u];
                        }
#pragma unroll
                        for (int q = 0; q < RU; ++q) {
                            const int64_t r = r0 + q * kBlock;
                            if (r >= rows) break;
                            if (keep) Gk[r] = sum[q];
                            const float v = (float)(sum[q] / (double)nk);
                            Ck[r] = v;
                            a += (double)v * (double)v;
                        }
                    }
                }
            } else {
                for (int64_t r = threadIdx.x; r < rows; r += kBlock) {
                    const double x = (double)Ck[r];
                    a += x * x;
                }
            }
            block_sum3(a, zb, zc);
            if (threadIdx.x == 0) B.cnorm[k] = a;
        });
        if (!grid_sync(gs, nb, tmo, BP_FINALIZE, tclk)) return;
        // D: the fused ALM sweep (instances starting an outer iteration), walked over
        //    the group segments; it also leaves the next L-step's group sums in pmeans
        load_tab(A.off_seg);
        for_items(batch, s_tab, s_mode, [](int m, int) { return m == M_ITER; }, [&](int i, int local) {
            BatchInst& B = inst[i];
            const int sg = local / B.mrb, rb = local % B.mrb;
            const int64_t r0 = (int64_t)rb * kBatchRows;
            if (sg >= s_nseg[i] || r0 >= B.dp) {   // no segment or rows here: zero partials only
                if (threadIdx.x < 3) B.sweep_part[3 * local + threadIdx.x] = 0.0;
                return;
            }
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            {
                const double rho = B.rho;
                const double alpha = rho / (2.0 * B.lambda + rho);
                const double beta = (2.0 * B.lambda) / (2.0 * B.lambda + rho);
                const double next = B.kappa * rho;
                const double inv_next = 1.0 / (next < B.rho_max ? next : B.rho_max);
                const int begin = B.segb[sg];
                seg_sweep_tile<float, 4, kBatchRows, 4, 2, false, true>(   // compact l1 state in S
                    B.X, B.dp, B.L, B.dp, B.S, B.dp, nullptr, 0, B.C, B.lab[B.cur][B.perm[begin]], B.dp,
                    B.perm, begin, B.segl[sg], r0, (float)alpha, (float)beta, (float)rho,
                    (float)(1.0 / rho), (float)inv_next, a0, a1, a2, B.pmeans + (int64_t)sg * B.dp,
                    nullptr, (float)B.rho_prev, (float)(1.0 / B.rho_prev));
            }
            block_sum3(a0, a1, a2);
            if (threadIdx.x == 0) {
                B.sweep_part[3 * local] = a0;
                B.sweep_part[3 * local + 1] = a1;
                B.sweep_part[3 * local + 2] = a2;
            }
        });
        if (!grid_sync(gs, nb, tmo, BP_SWEEP, tclk)) return;
        // F: distance tiles (columns of X before the iterations, of L after)
        load_tab(A.off_dist);
        for_items(batch, s_tab, s_mode, assigns, [&](int i, int local) {
            BatchInst& B = inst[i];
            const int mode = s_mode[i];
            const int kc = local % B.nkc, ts = local / B.nkc;
            const int tile = ts / B.slices, s = ts % B.slices;
            const int rows = mode_rows(B, mode);
            dist_tile<true, false>(B.C, rows, B.c, B.kpad, kmeans_matrix(B, mode), rows, B.n,
                                   B.slice_rows, B.part, nullptr, (int64_t)tile * kJT, s, kc * kKC,
                                   false);
        });
        if (!grid_sync(gs, nb, tmo, BP_DIST, tclk)) return;
        // G: reduce slices, argmin (16 lanes per column; lane group g of an item takes
        //    its columns g, g + 16, ...), changed counts
        load_tab(A.off_col);
        for_items(batch, s_tab, s_mode, assigns, [&](int i, int local) {
            BatchInst& B = inst[i];
            const int q = threadIdx.x & 15;
            constexpr int NJ = kArgminCols / 16;
            int64_t j[NJ], jc[NJ];   // jc: clamped into the matrix (results past n dropped)
#pragma unroll
            for (int c2 = 0; c2 < NJ; ++c2) {
                j[c2] = (int64_t)local * (16 * NJ) + 16 * c2 + (threadIdx.x >> 4);
                jc[c2] = j[c2] < B.n ? j[c2] : B.n - 1;
            }
            double bestd[NJ];
            int bestk[NJ];
#pragma unroll
            for (int c2 = 0; c2 < NJ; ++c2) { bestd[c2] = INFINITY; bestk[c2] = INT_MAX; }
            const int ns = B.slices;
            // 64 groups per chunk; every column's loads of four slices are issued
            // before their additions (each column's slices added in slice order)
            for (int k0 = 0; k0 < B.c; k0 += 64) {
                double dot[NJ][4];
#pragma unroll
                for (int c2 = 0; c2 < NJ; ++c2)
#pragma unroll
                    for (int t = 0; t < 4; ++t) dot[c2][t] = 0.0;
                for (int s0 = 0; s0 < ns; s0 += 4) {
                    float v[NJ][4][4];
#pragma unroll
                    for (int c2 = 0; c2 < NJ; ++c2)
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int su = s0 + u < ns ? s0 + u : ns - 1;
                            const float* pp = B.part + ((int64_t)su * B.n + jc[c2]) * B.kpad;
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                const int k = k0 + q + 16 * t;
                                v[c2][u][t] = pp[k < B.kpad ? k : B.kpad - 1];
                            }
                        }
#pragma unroll
                    for (int c2 = 0; c2 < NJ; ++c2)
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int t = 0; t < 4; ++t)
                                dot[c2][t] += (s0 + u < ns && k0 + q + 16 * t < B.c) ? (double)v[c2][u][t] : 0.0;
                }
                double cn[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = k0 + q + 16 * t;
                    cn[t] = B.cnorm[k < B.c ? k : B.c - 1];
                }
#pragma unroll
                for (int c2 = 0; c2 < NJ; ++c2)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int k = k0 + q + 16 * t;
                        if (k < B.c) {
                            const double dist = cn[t] - 2.0 * dot[c2][t];
                            if (dist < bestd[c2]) { bestd[c2] = dist; bestk[c2] = k; }
                        }
                    }
            }
            int wch = 0;
#pragma unroll
            for (int c2 = 0; c2 < NJ; ++c2) {
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) {
                    const double od = __shfl_xor(bestd[c2], o, 16);
                    const int ok = __shfl_xor(bestk[c2], o, 16);
                    if (od < bestd[c2] || (od == bestd[c2] && ok < bestk[c2])) { bestd[c2] = od; bestk[c2] = ok; }
                }
                bool moved = false;
                if (j[c2] < B.n && q == 0) {
                    const int lab = bestk[c2] == INT_MAX ? 0 : bestk[c2];
                    B.lab[B.cur ^ 1][j[c2]] = lab;
                    moved = B.lab[B.cur][j[c2]] != lab;
                }
                wch += __popcll(__ballot(moved));
            }
            // changed count per wave (no workgroup barrier): chg[4 item + wave]
            if ((threadIdx.x & 63) == 0) B.chg[4 * local + (threadIdx.x >> 6)] = wch;
        });
        if (!grid_sync(gs, nb, tmo, BP_ARGMIN, tclk)) return;
        // H: control
        for (int i = blockIdx.x; i < batch; i += nb) {
            control_instance(inst[i], active);
            __syncthreads();
        }
        if (threadIdx.x == 0 && blockIdx.x == 0) gs->steps += 1;
        if (!grid_sync(gs, nb, tmo, BP_CONTROL, tclk)) return;
    }

    // ---- results: L, S = soft(B, 1/rho of the last sweep) (first d rows) and labels
    //      into the caller's buffers
    load_tab(A.off_tile);
    for (int t = threadIdx.x; t < batch; t += kBlock) s_mode[t] = 1;
    __syncthreads();
    for_items(batch, s_tab, s_mode, any, [&](int i, int local) {
        BatchInst& B = inst[i];
        if (B.status < 0) return;
        const int cb = local / B.nrb, rb = local % B.nrb;
        const int64_t j0 = (int64_t)cb * B.jc, j1 = min((int64_t)B.n, j0 + B.jc);
        const int64_t r0 = (int64_t)rb * kBatchRows;
        const int64_t r1 = min((int64_t)B.d, r0 + kBatchRows);
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;   // wave per column
        const float tau = (float)(1.0 / B.rho_prev);
        for (int64_t j = j0 + w; j < j1; j += kBlock / 64)
            for (int64_t r = r0 + lane; r < r1; r += 64) {
                B.Lc[j * B.ldl + r] = B.L[j * B.dp + r];
                B.Sc[j * B.lds + r] = soft_threshold(B.S[j * B.dp + r], tau);
            }
    });
    for (int i = blockIdx.x; i < batch; i += nb) {
        BatchInst& B = inst[i];
        if (B.labels_out && B.status >= 0) {
            const int32_t* src = B.lab[B.cur];
            for (int j = threadIdx.x; j < B.n; j += kBlock) B.labels_out[j] = src[j];
        }
    }
}

__global__ void k_batched_reset(BatchSync* s, int batch) {
    if (threadIdx.x == 0) {
        s->count = 0u;
        s->gen = 0u;
        s->abort = 0;
        s->active = batch;
        s->steps = 0;
    }
    if (threadIdx.x < BP_COUNT) s->phase_ticks[threadIdx.x] = 0;
    for (int t = threadIdx.x; t < 8 * 64; t += blockDim.x) s->group_count[t] = 0u;
}

}  // namespace

void launch_batched_reset(BatchSync* s, int batch, hipStream_t st) {
    k_batched_reset<<<1, 64, 0, st>>>(s, batch);
}

void launch_batched(const BatchArgs& args, int nblocks, hipStream_t st) {
    k_batched<<<nblocks, kBlock, 0, st>>>(args);
}

int batched_blocks_per_cu() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched, kBlock, 0) != hipSuccess)
        return 0;
    return blocks;
}

}  // namespace respca
