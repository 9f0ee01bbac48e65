// gfx950 kernels of librespca: the per-iteration RES-PCA sweep and its K-means.
//
// Layout: every d x n matrix is column-major; a streaming workgroup owns a
// slice of kRowsPerBlock consecutive rows and walks columns, so each wave64
// load touches 64 consecutive rows of one column (coalesced), vectorised to
// 16-byte loads when d and the leading dimensions allow it.  All reductions
// are two-level (workgroup partials, then one fixed-order pass), so results
// are bitwise reproducible run to run; no floating-point atomics are used.
#include "kernels.h"
#include "device_common.h"

static_assert(respca::kSegCols <= respca::kMaxSegCols, "segments must fit the LDS column list");

#include <hip/hip_runtime.h>

#include <climits>
#include <algorithm>
#include <cmath>

namespace respca {

namespace {

// Vector width usable for a set of column-major operands: 16-byte accesses
// need d and every leading dimension to be multiples of the width and 16-byte
// aligned bases, so that a vector never straddles a column end.
template <typename T>
inline int pick_vec(int64_t d, std::initializer_list<std::pair<const void*, int64_t>> ops) {
    constexpr int V = 16 / sizeof(T);
    if (d % V) return 1;
    for (auto& o : ops) {
        if (o.second % V) return 1;
        if (reinterpret_cast<uintptr_t>(o.first) % 16) return 1;
    }
    return V;
}

// ------------------------------------------------------------------ fills

template <typename T>
__global__ void k_zero2d(T* A, int64_t ld, int64_t d, int64_t n) {
    const int64_t total = d * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / d, i = e - j * d;
        A[j * ld + i] = T(0);
    }
}

__global__ void k_zero_i32(int32_t* a, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        a[e] = 0;
}

// ----------------------------------------------------------- sum of squares

// Workgroup (cb, rb): columns [cb*jc, cb*jc + jc) of row slice rb.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sumsq(const T* X, int64_t ldx, int64_t d, int64_t n,
                                                  int jc, double* partial) {
    const int64_t r0 = (int64_t)blockIdx.y * kRowsPerBlock;
    const int64_t j0 = (int64_t)blockIdx.x * jc;
    const int64_t j1 = j0 + jc < n ? j0 + jc : n;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t j = j0; j < j1; ++j)
        for (int s = 0; s < kRowsPerBlock / kBlock; ++s) {
            const int64_t i = r0 + s * kBlock + threadIdx.x;
            if (i < d) { const double x = (double)X[j * ldx + i]; a += x * x; }
        }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * gridDim.y + blockIdx.y] = a;
}

// One workgroup; `width` interleaved sums over `count` records, fixed order.
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* partial, int count,
                                                         int width, double* out) {
    for (int w = 0; w < width; ++w) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int r = threadIdx.x; r < count; r += kBlock) a += partial[(int64_t)r * width + w];
        block_sum3(a, b, c);
        if (threadIdx.x == 0) out[w] = a;
        __syncthreads();
    }
}

// --------------------------------------------------------------- label sort

// Stable counting sort in three launches.  Chunk b = columns [256b, 256b+256):
//   hist:    per-chunk label histogram -> bc[b*c + k]
//   scan:    per label, exclusive offsets over (label, chunk) -> bc in place;
//            group counts and the segment table (runs of <= kSegCols columns)
//   scatter: each column's rank among equal labels earlier in its chunk.
// Output order: by label, then by column index.
constexpr int kSortChunk = 256;

__global__ __launch_bounds__(kSortChunk) void k_sort_hist(const int32_t* __restrict__ labels, int n,
                                                          int c, int32_t* __restrict__ bc) {
    __shared__ int h[kMaxGroups];
    for (int k = threadIdx.x; k < c; k += kSortChunk) h[k] = 0;
    __syncthreads();
    const int j = blockIdx.x * kSortChunk + threadIdx.x;
    if (j < n) atomicAdd(&h[labels[j]], 1);
    __syncthreads();
    for (int k = threadIdx.x; k < c; k += kSortChunk) bc[(int64_t)blockIdx.x * c + k] = h[k];
}

__device__ inline int block_exscan_1024(int v, int* wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
}

__global__ __launch_bounds__(kMaxGroups) void k_sort_scan(int32_t* __restrict__ bc, int nb, int c,
                                                         int32_t* counts, int32_t* seg_begin,
                                                         int32_t* seg_len, int32_t* seg_first,
                                                         int32_t* nseg_out) {
    __shared__ int wsum[kMaxGroups / 64];
    const int k = threadIdx.x;
    constexpr int U = 8;   // block counts loaded per step (independent loads in flight)
    int tot = 0;
    if (k < c)
        for (int b = 0; b < nb; b += U) {
            int v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = b + u < nb ? bc[(int64_t)(b + u) * c + k] : 0;
#pragma unroll
            for (int u = 0; u < U; ++u) tot += v[u];
        }
    const int nsg = (tot + kSegCols - 1) / kSegCols;
    const int base = block_exscan_1024(tot, wsum);
    const int sbase = block_exscan_1024(nsg, wsum);
    if (k < c) {
        counts[k] = tot;
        seg_first[k] = sbase;
        for (int q = 0; q < nsg; ++q) {
            seg_begin[sbase + q] = base + q * kSegCols;
            seg_len[sbase + q] = min(kSegCols, tot - q * kSegCols);
        }
        int run = base;
        for (int b = 0; b < nb; b += U) {
            int v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = b + u < nb ? bc[(int64_t)(b + u) * c + k] : 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b + u < nb) bc[(int64_t)(b + u) * c + k] = run;
                run += v[u];
            }
        }
        if (k == c - 1) { seg_first[c] = sbase + nsg; *nseg_out = sbase + nsg; }
    }
}

__global__ __launch_bounds__(kSortChunk) void k_sort_scatter(const int32_t* __restrict__ labels,
                                                             int n, int c,
                                                             const int32_t* __restrict__ bc,
                                                             int32_t* __restrict__ perm) {
    __shared__ int lab[kSortChunk];
    const int tid = threadIdx.x;
    const int j = blockIdx.x * kSortChunk + tid;
    const int my = j < n ? labels[j] : -1;
    lab[tid] = my;
    __syncthreads();
    if (j < n) {
        int rank = 0;
        for (int t = 0; t < tid; ++t) rank += (lab[t] == my);
        perm[bc[(int64_t)blockIdx.x * c + my] + rank] = j;
    }
}

// ---------------------------------------------------------- group partials

// Grid (segment slots, row slices); slots past the real segment count exit.
// COMPACT: S holds the compact state B (penalty rho_prev); Th is not read.
template <typename T, int V, bool WITH_D, bool COMPACT = false, bool NT = false>
__global__ __launch_bounds__(kBlock) void k_group_partial(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ S, int64_t lds,
    const T* __restrict__ Th, int64_t ldt, T inv_rho, int64_t d, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ seg_begin, const int32_t* __restrict__ seg_len,
    const int32_t* __restrict__ nseg, int nrb, double* __restrict__ partial, T rho_prev = T(0),
    T inv_rho_prev = T(0)) {
    const int s = (int)(blockIdx.x / nrb);   // row blocks vary fastest
    if (s >= *nseg) return;
    group_partial_tile<T, V, WITH_D, kRowsPerBlock, 1, COMPACT, NT>(
        A, lda, S, lds, Th, ldt, inv_rho, d, perm, seg_begin[s], seg_len[s],
        (int64_t)(blockIdx.x % nrb) * kRowsPerBlock, partial + (int64_t)s * d, rho_prev, inv_rho_prev);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_group_finalize(const double* __restrict__ partial,
                                                           int64_t d, const int32_t* counts,
                                                           const int32_t* seg_first, T* C,
                                                           double* __restrict__ gsum) {
    const int k = blockIdx.y;
    const int nk = counts[k];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= d) return;
    if (nk == 0) {
        if (gsum) gsum[(int64_t)k * d + i] = 0.0;   // an empty group's sum is exactly zero
        return;
    }
    double s = 0.0;
    const int g1 = seg_first[k + 1];
    for (int g = seg_first[k]; g < g1; g += 4) {   // four loads in flight, added in segment order
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)                  // clamped: no branch per load
            v[u] = partial[(int64_t)(g + u < g1 ? g + u : g1 - 1) * d + i];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (g + u < g1) s += v[u];
    }
    if (gsum) gsum[(int64_t)k * d + i] = s;
    C[(int64_t)k * d + i] = (T)(s / (double)nk);
}

// -------------------------------------------------- incremental group means
//
// After an assignment pass that moved few columns, the group sums of Y follow
// from the previous ones: column j with new label b != old label a is listed
// under key b (entering b) and key c + a (leaving a).  A counting sort of these
// entries (keys in order, columns in order within a key) gives segments for the
// group-partial kernel, and the update adds each group's entering partials and
// subtracts its leaving partials, segment by segment in order.

__global__ __launch_bounds__(kSortChunk) void k_chg_hist(const int32_t* __restrict__ nl,
                                                         const int32_t* __restrict__ ol, int n,
                                                         int c, int32_t* __restrict__ bc) {
    __shared__ int h[2 * kMaxGroups];
    const int K = 2 * c;
    for (int k = threadIdx.x; k < K; k += kSortChunk) h[k] = 0;
    __syncthreads();
    const int j = blockIdx.x * kSortChunk + threadIdx.x;
    if (j < n) {
        const int a = ol[j], b = nl[j];
        if (a != b) {
            atomicAdd(&h[b], 1);
            atomicAdd(&h[c + a], 1);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kSortChunk) bc[(int64_t)blockIdx.x * K + k] = h[k];
}

// One workgroup of kMaxGroups threads, thread t owns keys 2t and 2t + 1 (of 2c):
// key totals, exclusive offsets (bc in place), the segment table (seg_first has
// 2c + 1 entries) and the new group counts counts_new[k] = counts_old[k] +
// entering(k) - leaving(k).
// Segments past max_seg (more moved columns than the tables were sized for) are
// not written and seg_first is clamped to max_seg.
__global__ __launch_bounds__(kMaxGroups) void k_chg_scan(int32_t* __restrict__ bc, int nb, int c,
                                                        const int32_t* __restrict__ counts_old,
                                                        int32_t* __restrict__ counts_new,
                                                        int32_t* __restrict__ seg_begin,
                                                        int32_t* __restrict__ seg_len,
                                                        int32_t* __restrict__ seg_first,
                                                        int32_t* __restrict__ nseg_out, int max_seg) {
    __shared__ int wsum[kMaxGroups / 64];
    __shared__ int tots[2 * kMaxGroups];
    const int K = 2 * c;
    const int t = threadIdx.x;
    constexpr int U = 8;
    int tot[2] = {0, 0};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int key = 2 * t + e;
        if (key < K)
            for (int b = 0; b < nb; b += U) {
                int v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = b + u < nb ? bc[(int64_t)(b + u) * K + key] : 0;
#pragma unroll
                for (int u = 0; u < U; ++u) tot[e] += v[u];
            }
    }
    const int nsg[2] = {(tot[0] + kSegCols - 1) / kSegCols, (tot[1] + kSegCols - 1) / kSegCols};
    const int base = block_exscan_1024(tot[0] + tot[1], wsum);
    const int sbase = block_exscan_1024(nsg[0] + nsg[1], wsum);
    int off = base, soff = sbase;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int key = 2 * t + e;
        if (key < K) {
            tots[key] = tot[e];
            seg_first[key] = min(soff, max_seg);
            for (int q = 0; q < nsg[e] && soff + q < max_seg; ++q) {
                seg_begin[soff + q] = off + q * kSegCols;
                seg_len[soff + q] = min(kSegCols, tot[e] - q * kSegCols);
            }
            int run = off;
            for (int b = 0; b < nb; b += U) {
                int v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = b + u < nb ? bc[(int64_t)(b + u) * K + key] : 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (b + u < nb) bc[(int64_t)(b + u) * K + key] = run;
                    run += v[u];
                }
            }
            if (key == K - 1) {
                seg_first[K] = min(soff + nsg[e], max_seg);
                *nseg_out = min(soff + nsg[e], max_seg);
            }
        }
        off += tot[e];
        soff += nsg[e];
    }
    __syncthreads();
    for (int k = t; k < c; k += kMaxGroups) counts_new[k] = counts_old[k] + tots[k] - tots[c + k];
}

__global__ __launch_bounds__(kSortChunk) void k_chg_scatter(const int32_t* __restrict__ nl,
                                                            const int32_t* __restrict__ ol, int n,
                                                            int c, const int32_t* __restrict__ bc,
                                                            int32_t* __restrict__ perm) {
    __shared__ int ek[kSortChunk], lk[kSortChunk];   // entering / leaving key, -1 if unchanged
    const int tid = threadIdx.x;
    const int j = blockIdx.x * kSortChunk + tid;
    const int a = j < n ? ol[j] : 0, b = j < n ? nl[j] : 0;
    const bool moved = j < n && a != b;
    ek[tid] = moved ? b : -1;
    lk[tid] = moved ? c + a : -1;
    __syncthreads();
    if (moved) {
        const int K = 2 * c;
        int re = 0, rl = 0;
        for (int t = 0; t < tid; ++t) {
            re += (ek[t] == b);
            rl += (lk[t] == c + a);
        }
        perm[bc[(int64_t)blockIdx.x * K + b] + re] = j;
        perm[bc[(int64_t)blockIdx.x * K + c + a] + rl] = j;
    }
}

// gsum[:, k] += (entering partials) - (leaving partials) for every group with
// moved columns; C[:, k] = gsum[:, k] / n_k (an emptied group keeps C[:, k] and
// its sum becomes exactly zero).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_group_update(const double* __restrict__ partial,
                                                         int64_t d, int c,
                                                         const int32_t* __restrict__ counts_new,
                                                         const int32_t* __restrict__ seg_first,
                                                         double* __restrict__ gsum, T* C,
                                                         int32_t* __restrict__ counts_out) {
    const int k = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x == 0) counts_out[k] = counts_new[k];
    const int e0 = seg_first[k], e1 = seg_first[k + 1];
    const int l0 = seg_first[c + k], l1 = seg_first[c + k + 1];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if ((e0 == e1 && l0 == l1) || i >= d) return;   // no column entered or left group k
    const int nk = counts_new[k];
    double* gk = gsum + (int64_t)k * d;
    if (nk == 0) {
        gk[i] = 0.0;
        return;
    }
    double add = 0.0, sub = 0.0;
    for (int g = e0; g < e1; ++g) add += partial[(int64_t)g * d + i];
    for (int g = l0; g < l1; ++g) sub += partial[(int64_t)g * d + i];
    const double sum = gk[i] + (add - sub);
    gk[i] = sum;
    C[(int64_t)k * d + i] = (T)(sum / (double)nk);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_col_sqnorm(const T* C, int64_t d, double* out) {
    const int k = blockIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += kBlock) {
        const double x = (double)C[(int64_t)k * d + i];
        a += x * x;
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) out[k] = a;
}

// ------------------------------------------------------------------- sweep

// The fused ALM sweep walked in group order (tile body seg_sweep_tile):
// workgroup (s, rb) takes segment s of the label sort (at most kSegCols columns
// of one group) over one row block, row blocks varying fastest so that resident
// workgroups share a band of segments.  Beside L, S, Theta and the norm partials
// it writes the group sums of D at the next penalty, which let the next
// iteration skip its means pass when the p-step keeps every label.  Slots past
// the segment count write zero norms.  L21: column-wise S-step from fac.
// COMPACT: the l1 sweep on the compact state B (kept in S, previous penalty
// rho_prev; Th is not used), see seg_sweep_tile.
template <typename T, int V, bool L21, bool COMPACT = false, int UU = 4, bool NT = false>
__global__ __launch_bounds__(kBlock) void k_sweep_seg(
    const T* __restrict__ X, int64_t ldx, T* __restrict__ L, int64_t ldl, T* __restrict__ S,
    int64_t lds, T* __restrict__ Th, int64_t ldt, const T* __restrict__ C,
    const int32_t* __restrict__ labels, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ seg_begin, const int32_t* __restrict__ seg_len,
    const int32_t* __restrict__ nseg, int64_t d, int nrb, T alpha, T beta, T rho, T inv_rho,
    T inv_rho_next, double* __restrict__ norm_partial, double* __restrict__ next_partial,
    const double* __restrict__ fac, T rho_prev = T(0), T inv_rho_prev = T(0)) {
    const int sg = (int)(blockIdx.x / nrb);
    const int64_t r0 = (int64_t)(blockIdx.x % nrb) * kRowsPerBlock;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (sg < *nseg) {
        const int begin = seg_begin[sg];
        seg_sweep_tile<T, V, kRowsPerBlock, 1, UU, L21, COMPACT, NT>(
            X, ldx, L, ldl, S, lds, Th, ldt, C, labels[perm[begin]], d, perm, begin, seg_len[sg], r0,
            alpha, beta, rho, inv_rho, inv_rho_next, a0, a1, a2, next_partial + (int64_t)sg * d, fac,
            rho_prev, inv_rho_prev);
    }
    block_sum3(a0, a1, a2);
    if (threadIdx.x == 0) {
        double* o = norm_partial + 3 * (int64_t)blockIdx.x;
        o[0] = a0; o[1] = a1; o[2] = a2;
    }
}

// ---------------------------------------------------------- l2,1 factors

// Column-wise S-step (l2,1 penalty), first half: a workgroup per column (grid
// stride over the columns) sums ||B_j||^2 in
// double over the column (fixed order: thread stride, then the block sum), with
// B_j formed in T exactly as the sweep forms it, and stores the block soft
// threshold factor max(0, 1 - 1/(rho ||B_j||)).
template <typename T, int V, bool NT = false>
__global__ __launch_bounds__(kBlock) void k_l21_factor(
    const T* __restrict__ X, int64_t ldx, const T* __restrict__ S, int64_t lds,
    const T* __restrict__ Th, int64_t ldt, const T* __restrict__ C,
    const int32_t* __restrict__ labels, int64_t d, int64_t n, T alpha, T beta, T inv_rho,
    double rho, double* __restrict__ fac) {
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        const T* x = X + j * ldx;
        const T* s = S + j * lds;
        const T* t = Th + j * ldt;
        const T* m = C + (int64_t)labels[j] * d;
        double a = 0.0, b0 = 0.0, c0 = 0.0;
        for (int64_t i = (int64_t)threadIdx.x * V; i < d; i += (int64_t)kBlock * V) {
            T xs[V], ss[V], ts[V], ms[V];
            sload<NT, T, V>(x + i, xs);
            sload<NT, T, V>(s + i, ss);
            sload<NT, T, V>(t + i, ts);
            vload<T, V>(m + i, ms);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const T dv = xs[v] - ss[v] + ts[v] * inv_rho;
                const T ln = alpha * dv + beta * ms[v];
                const T b = xs[v] - ln + ts[v] * inv_rho;
                a += (double)b * (double)b;
            }
        }
        block_sum3(a, b0, c0);   // uniform over the block; safe to repeat per column
        if (threadIdx.x == 0) {
            const double nb = sqrt(a);
            fac[j] = rho * nb > 1.0 ? 1.0 - 1.0 / (rho * nb) : 0.0;
        }
    }
}

// -------------------------------------------------------------------- dots

// Tile: 64 columns x CT = 16*KB groups, over one slice of slice_rows rows,
// staged through LDS 32 rows at a time; each thread owns a KB x 4 block.
template <typename T, int KB>
__global__ __launch_bounds__(kBlock) void k_dots(const T* __restrict__ C, int64_t d, int c,
                                                 const T* __restrict__ Y, int64_t ldy, int64_t n,
                                                 int64_t slice_rows, T* __restrict__ part) {
    constexpr int CT = 16 * KB, JT = 64, RT = 32;
    __shared__ T As[RT][CT + 4];
    __shared__ T Bs[RT][JT + 4];
    const int tid = threadIdx.x, tk = tid >> 4, tj = tid & 15;
    const int64_t j0 = (int64_t)blockIdx.x * JT;
    const int k0 = blockIdx.y * CT;
    const int rb = blockIdx.z;
    const int64_t rbeg = (int64_t)rb * slice_rows;
    const int64_t rend = rbeg + slice_rows < d ? rbeg + slice_rows : d;
    T acc[KB][4];
#pragma unroll
    for (int a = 0; a < KB; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = T(0);

    for (int64_t r = rbeg; r < rend; r += RT) {
#pragma unroll
        for (int m = 0; m < (RT * JT) / kBlock; ++m) {
            const int e = tid + kBlock * m, row = e & (RT - 1), col = e / RT;
            const int64_t gi = r + row, gj = j0 + col;
            Bs[row][col] = (gi < rend && gj < n) ? Y[gj * ldy + gi] : T(0);
        }
#pragma unroll
        for (int m = 0; m < (RT * CT) / kBlock; ++m) {
            const int e = tid + kBlock * m, row = e & (RT - 1), col = e / RT;
            const int64_t gi = r + row;
            const int gk = k0 + col;
            As[row][col] = (gi < rend && gk < c) ? C[(int64_t)gk * d + gi] : T(0);
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < RT; ++rr) {
            T a[KB], b[4];
#pragma unroll
            for (int q = 0; q < KB; ++q) a[q] = As[rr][tk * KB + q];
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = Bs[rr][tj * 4 + q];
#pragma unroll
            for (int x = 0; x < KB; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < KB; ++x) {
        const int k = k0 + tk * KB + x;
        if (k >= c) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int64_t j = j0 + tj * 4 + y;
            if (j < n) part[((int64_t)rb * c + k) * n + j] = acc[x][y];
        }
    }
}

// Sixteen lanes per column: lane q scores groups q, q + 16, ... (slices summed in
// order), then the lanes keep the smallest distance, the lowest group on ties.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_argmin(const T* __restrict__ part, int nrb, int c,
                                                   int64_t n, const double* __restrict__ cnorm,
                                                   const int32_t* __restrict__ old_labels,
                                                   int32_t* __restrict__ new_labels,
                                                   double* __restrict__ changed_partial) {
    const int q = threadIdx.x & 15;
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool live = j < n;
    double bestd = INFINITY;
    int bestk = INT_MAX;
    if (live)
        for (int k = q; k < c; k += 16) {
            // eight slices' loads issued together (indices clamped, the extra values
            // not added), then added in slice order
            double dot = 0.0;
            for (int rb0 = 0; rb0 < nrb; rb0 += 8) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int rb = rb0 + u < nrb ? rb0 + u : nrb - 1;
                    v[u] = part[((int64_t)rb * c + k) * n + j];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (rb0 + u < nrb) dot += (double)v[u];
            }
            const double dist = cnorm[k] - 2.0 * dot;
            if (dist < bestd) { bestd = dist; bestk = k; }
        }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        const double od = __shfl_xor(bestd, o, 16);
        const int ok = __shfl_xor(bestk, o, 16);
        if (od < bestd || (od == bestd && ok < bestk)) { bestd = od; bestk = ok; }
    }
    double changed = 0.0;
    if (live && q == 0) {
        const int best = bestk == INT_MAX ? 0 : bestk;
        new_labels[j] = best;
        changed = (old_labels[j] != best) ? 1.0 : 0.0;
    }
    double b = 0.0, c2 = 0.0;
    block_sum3(changed, b, c2);
    if (threadIdx.x == 0) changed_partial[blockIdx.x] = changed;
}

// -------------------------------------------------------------- k-means++

// One wave per column: d2[j] = min(d2[j], ||Y_j - Y_s||^2) in double, s = seeds[m]
// (the differences of the upcast values are taken in double as well).
// k-means++ D^2 update (Sec. 4.2 initialisation): d2[j] = min(d2[j], ||y_j - y_s||^2)
// for the newest seed s = seeds[m] (m = 0: the first distances).  One wave per column.
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_d2(const T* __restrict__ Y, int64_t ldy, int64_t d,
                                               int64_t n, const int32_t* __restrict__ seeds, int m,
                                               double* __restrict__ d2) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (j >= n) return;
    const double acc = d2_column<T, V>(Y + j * ldy, Y + (int64_t)seeds[m] * ldy, d, lane);
    if (lane == 0) d2[j] = (m == 0) ? acc : fmin(d2[j], acc);
}

// Half-precision copy for bounded seeding (float runs).  Column j is stored as
// z = y_j / sc_j in fp16, sc_j the power of two that puts max |y_j| in
// [2^14, 2^15) (at least 2^-126), so |z sc_j - y_j| <= 2^-11 |y_j| + 2^-25 sc_j
// per element; Z has ldz >= d rows, zero past row d.  This first pass also
// computes the exact distances to seed 0 and the column norms.
template <int V>
__global__ __launch_bounds__(kBlock) void k_d2_first(const float* __restrict__ Y, int64_t ldy,
                                                     int64_t d, int64_t n,
                                                     const int32_t* __restrict__ seeds,
                                                     double* __restrict__ d2, _Float16* __restrict__ Z,
                                                     int64_t ldz, float* __restrict__ zsc,
                                                     double* __restrict__ ynorm) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (j >= n) return;
    const float* yj = Y + j * ldy;
    double nn = 0.0;
    float mx = 0.f;
    const double acc = d2_column<float, V, true>(yj, Y + (int64_t)seeds[0] * ldy, d, lane, &nn, &mx);
    nn = wave_sum(nn);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    int e = mx > 0.f ? ilogbf(mx) - 14 : 0;
    if (e < -126) e = -126;
    const float inv = ldexpf(1.f, -e);   // exact: z = y * 2^-e
    _Float16* zj = Z + j * ldz;
    typedef _Float16 half4 __attribute__((ext_vector_type(4)));
    for (int64_t i = (int64_t)lane * 4; i < ldz; i += 256) {   // ldz % 8 == 0: 8-byte stores
        float x[4];
        if (V == 4 && i + 4 <= d) {
            vload<float, 4>(yj + i, x);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = i + e < d ? yj[i + e] : 0.f;
        }
        half4 z;
#pragma unroll
        for (int e = 0; e < 4; ++e) z[e] = (_Float16)(x[e] * inv);
        *reinterpret_cast<half4*>(zj + i) = z;
    }
    if (lane == 0) {
        d2[j] = acc;
        ynorm[j] = sqrt(nn);
        zsc[j] = ldexpf(1.f, e);
    }
}

// Bounded D^2 update for seeds m >= 1 (float runs).  A lower bound on
// ||y_j - y_s|| comes from the fp16 copies of both columns: sqrt(A / (1 + eta)) -
// E_j - E_s, with A the FP32 sum of (z_j,i sc_j - z_s,i sc_s)^2 (relative error at
// most eta; z_s,i sc_s is exact up to underflow, below 2^-149 per row) and E_j =
// 2^-10 ||y_j|| + 2^-24 sc_j sqrt(d) a copy's error bound (twice the rounding
// bound), E_s the seed copy's, plus sqrt(d) 2^-149.  When the bound already exceeds
// d2[j] the minimum cannot change and the exact distance is skipped; otherwise it
// is computed exactly as in k_d2, so d2 holds the same values either way.  Reading
// the seed's copy instead of its FP32 column halves what each pass takes from the
// caches for the seed.
template <int V>
__global__ __launch_bounds__(kBlock) void k_d2_bounded(const float* __restrict__ Y, int64_t ldy,
                                                       int64_t d, int64_t n,
                                                       const int32_t* __restrict__ seeds, int m,
                                                       double* __restrict__ d2,
                                                       const _Float16* __restrict__ Z, int64_t ldz,
                                                       const float* __restrict__ zsc,
                                                       const double* __restrict__ ynorm, float eta) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (j >= n) return;
    const int64_t sd = seeds[m];
    const float* ys = Y + sd * ldy;
    const _Float16* zj = Z + j * ldz;
    const _Float16* zs = Z + sd * ldz;
    const float sc = zsc[j], scs = zsc[sd];
    typedef _Float16 half8 __attribute__((ext_vector_type(8)));
    float acc = 0.f;
    int64_t i = (int64_t)lane * 8;
    // whole 512-row passes, four at a time: their loads are issued before any of
    // their arithmetic (the same additions in the same order as below)
    constexpr int U = 4;
    const int64_t nfull = d / 512;
    for (int64_t t = 0; t + U <= nfull; t += U, i += 512 * U) {
        half8 z[U], w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            z[u] = *reinterpret_cast<const half8*>(zj + i + 512 * u);
            w[u] = *reinterpret_cast<const half8*>(zs + i + 512 * u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float t2 = fmaf((float)z[u][e], sc, -((float)w[u][e] * scs));
                acc = fmaf(t2, t2, acc);
            }
    }
    for (; i < ldz; i += 512) {   // ldz % 8 == 0: 16-byte loads; both copies are zero past row d
        const half8 z = *reinterpret_cast<const half8*>(zj + i);
        const half8 w = *reinterpret_cast<const half8*>(zs + i);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float t = fmaf((float)z[e], sc, -((float)w[e] * scs));
            acc = fmaf(t, t, acc);
        }
    }
    // A less the largest total of underflowed squares (2^-148 per term), then the
    // relative error; an infinite or NaN A never skips
    const double A = wave_sum((double)acc) - (double)ldz * ldexp(1.0, -148);
    const double rd = sqrt((double)d);
    const double E = (ldexp(1.0, -10) * (ynorm[j] + ynorm[sd]) +
                      ldexp(1.0, -24) * ((double)sc + (double)scs) * rd + ldexp(1.0, -149) * rd) *
                     (1.0 + 1e-6);
    const double lb = sqrt(fmax(A, 0.0) / (1.0 + (double)eta)) - E;
    const double cur = d2[j];
    if (isfinite(A) && lb > 0.0 && lb * lb * (1.0 - 1e-9) > cur) return;   // the minimum stays cur
    const double ex = d2_column<float, V>(Y + j * ldy, ys, d, lane);
    if (lane == 0) d2[j] = fmin(cur, ex);
}

__device__ inline int block_min_i(int v, int* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    int r = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = min(r, sh[i]);
    return r;
}

// Inverse-CDF draw of the next seed: thread t sums a contiguous chunk, a block
// scan gives each chunk its starting running sum, and the first index whose
// running sum exceeds u*total wins.  Chunks of at most kPickReg entries are
// loaded once, all loads issued together, and kept in registers for the search.
constexpr int kPickReg = 16;

__global__ __launch_bounds__(kPickThreads) void k_pick(const double* __restrict__ d2, int64_t n,
                                                       const double* __restrict__ u, int m,
                                                       int32_t* seeds, int32_t* chosen) {
    __shared__ double wtot[kPickThreads / 64];
    __shared__ int ish[kPickThreads / 64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t chunk = (n + kPickThreads - 1) / kPickThreads;
    const int64_t lo = tid * chunk, hi = lo + chunk < n ? lo + chunk : n;
    const bool inreg = chunk <= kPickReg;   // uniform
    double v[kPickReg];
    double loc = 0.0;
    if (inreg) {
#pragma unroll
        for (int e = 0; e < kPickReg; ++e) v[e] = lo + e < hi ? d2[lo + e] : 0.0;
#pragma unroll
        for (int e = 0; e < kPickReg; ++e)
            if (lo + e < hi) loc += v[e];
    } else {
        for (int64_t j = lo; j < hi; ++j) loc += d2[j];
    }
    double x = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    double pre = 0.0, total = 0.0;
    for (int w = 0; w < kPickThreads / 64; ++w) {
        if (w < wave) pre += wtot[w];
        total += wtot[w];
    }
    pre += x - loc;
    int s;
    if (total > 0.0) {
        const double target = u[m] * total;
        int cand = INT_MAX;
        double run = pre;
        if (inreg) {
#pragma unroll
            for (int e = 0; e < kPickReg; ++e)
                if (lo + e < hi && cand == INT_MAX) {
                    run += v[e];
                    if (run > target) cand = (int)(lo + e);
                }
        } else {
            for (int64_t j = lo; j < hi; ++j) {
                run += d2[j];
                if (run > target) { cand = (int)j; break; }
            }
        }
        s = block_min_i(cand, ish);
        if (s == INT_MAX) {
            int last = INT_MAX;  // largest index with a non-zero weight, via min of -j
            for (int64_t j = hi - 1; j >= lo; --j)
                if (d2[j] > 0.0) { last = -(int)j; break; }
            s = -block_min_i(last, ish);
        }
    } else {
        int cand = INT_MAX;
        for (int64_t j = lo; j < hi; ++j)
            if (!chosen[j]) { cand = (int)j; break; }
        s = block_min_i(cand, ish);
    }
    if (tid == 0) { seeds[m] = s; chosen[s] = 1; }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_cols(const T* __restrict__ Y, int64_t ldy,
                                                        int64_t d, const int32_t* __restrict__ idx,
                                                        T* __restrict__ C) {
    const int k = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < d) C[(int64_t)k * d + i] = Y[(int64_t)idx[k] * ldy + i];
}

inline int grid_cap(int64_t work, int per) {
    int64_t g = (work + per - 1) / per;
    if (g > 65535) g = 65535;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

// ================================================================ launchers

template <typename T>
void launch_zero2d(T* A, int64_t ld, int64_t d, int64_t n, hipStream_t st) {
    k_zero2d<T><<<grid_cap(d * n, kBlock * 8), kBlock, 0, st>>>(A, ld, d, n);
}

void launch_zero_f64(double* a, hipStream_t st) { k_zero2d<double><<<1, 64, 0, st>>>(a, 1, 1, 1); }

void launch_zero_i32(int32_t* a, int64_t count, hipStream_t st) {
    k_zero_i32<<<grid_cap(count, kBlock * 8), kBlock, 0, st>>>(a, count);
}

template <typename T>
int launch_sumsq(const T* X, int64_t ldx, int64_t d, int64_t n, double* partial, hipStream_t st) {
    const int nrb = row_blocks(d);
    const int jc = 16;
    const int ncb = (int)((n + jc - 1) / jc);
    k_sumsq<T><<<dim3(ncb, nrb), kBlock, 0, st>>>(X, ldx, d, n, jc, partial);
    return nrb * ncb;
}

// End of an assignment pass: out[0] = changed labels (partials + refined), out[1]
// = refined columns (0 without a refinement list).
__global__ __launch_bounds__(kBlock) void k_assign_finish(const double* partial, int count,
                                                          const int* counters, double* out,
                                                          StatusPublish pub) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int r = threadIdx.x; r < count; r += kBlock) a += partial[r];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) {
        const double changed = a + (counters ? (double)counters[1] : 0.0);
        const double refined = counters ? (double)counters[0] : 0.0;
        out[0] = changed;
        if (pub.seq == 0) {
            out[1] = refined;
            return;
        }
        out[1] = 0.0;
        volatile double* host = pub.host;
        for (int i = 0; i < 3; ++i) host[i] = pub.words[i];
        host[3] = changed;
        host[4] = refined;
        __threadfence_system();
        *(volatile uint64_t*)pub.host_seq = pub.seq;
        __threadfence_system();
    }
}

void launch_assign_finish(const double* partial, int count, const int* counters, double* out,
                          hipStream_t st, const StatusPublish& pub) {
    k_assign_finish<<<1, kBlock, 0, st>>>(partial, count, counters, out, pub);
}

__global__ void k_add_int(const int* counter, double* out, int set) {
    if (threadIdx.x == 0) out[0] = (set ? 0.0 : out[0]) + (double)counter[0];
}

void launch_add_int(const int* counter, double* out, hipStream_t st, bool set) {
    k_add_int<<<1, 64, 0, st>>>(counter, out, set ? 1 : 0);
}

void launch_sum_partials(const double* partial, int count, int width, double* out,
                         hipStream_t st) {
    k_sum_partials<<<1, kBlock, 0, st>>>(partial, count, width, out);
}

int64_t sort_scratch_ints(int64_t n, int c) { return ((n + kSortChunk - 1) / kSortChunk) * (int64_t)c; }

void launch_label_sort(const int32_t* labels, int64_t n, int c, int32_t* bc, int32_t* counts,
                       int32_t* perm, int32_t* seg_begin, int32_t* seg_len, int32_t* seg_first,
                       int32_t* nseg, hipStream_t st) {
    const int nb = (int)((n + kSortChunk - 1) / kSortChunk);
    k_sort_hist<<<nb, kSortChunk, 0, st>>>(labels, (int)n, c, bc);
    k_sort_scan<<<1, kMaxGroups, 0, st>>>(bc, nb, c, counts, seg_begin, seg_len, seg_first, nseg);
    k_sort_scatter<<<nb, kSortChunk, 0, st>>>(labels, (int)n, c, bc, perm);
}

// Whole passes over d x n arrays of at least this many bytes each load and store
// them nontemporally (see sload): such arrays exceed what the caches keep between
// passes, while small ones (a 500 x 500 problem) are faster cached.
constexpr double kStreamNtBytes = 64.0 * 1024 * 1024;

template <typename T>
bool stream_nt(int64_t d, int64_t n) {
    return (double)d * (double)n * sizeof(T) >= kStreamNtBytes;
}

template <typename T>
void launch_group_partial(bool with_d, const T* A, int64_t lda, const T* S, int64_t lds,
                          const T* Th, int64_t ldt, T inv_rho, int64_t d, int64_t n, int c,
                          const int32_t* perm, const int32_t* seg_begin, const int32_t* seg_len,
                          const int32_t* nseg, double* partial, hipStream_t st, int max_seg) {
    const int nrb = row_blocks(d);
    const unsigned grid = (unsigned)(max_seg >= 0 ? max_seg : max_segments(n, c)) * (unsigned)nrb;
    if (grid == 0) return;
    int v = with_d ? pick_vec<T>(d, {{A, lda}, {S, lds}, {Th, ldt}}) : pick_vec<T>(d, {{A, lda}});
    constexpr int VV = 16 / sizeof(T);
    // a whole pass (not the moved columns only) over large arrays: nontemporal
    const bool nt = max_seg < 0 && stream_nt<T>(d, n);
    const T* S2 = with_d ? S : A;
    const T* Th2 = with_d ? Th : A;
    const int64_t lds2 = with_d ? lds : lda, ldt2 = with_d ? ldt : lda;
    auto go = [&](auto kern) {
        kern<<<grid, kBlock, 0, st>>>(A, lda, S2, lds2, Th2, ldt2, inv_rho, d, perm, seg_begin,
                                      seg_len, nseg, nrb, partial, T(0), T(0));
    };
    if (with_d) {
        if (v == VV) nt ? go(k_group_partial<T, VV, true, false, true>) : go(k_group_partial<T, VV, true>);
        else nt ? go(k_group_partial<T, 1, true, false, true>) : go(k_group_partial<T, 1, true>);
    } else {
        if (v == VV) nt ? go(k_group_partial<T, VV, false, false, true>) : go(k_group_partial<T, VV, false>);
        else nt ? go(k_group_partial<T, 1, false, false, true>) : go(k_group_partial<T, 1, false>);
    }
}

template <typename T>
void launch_group_finalize(const double* partial, int64_t d, int c, const int32_t* counts,
                           const int32_t* seg_first, T* C, hipStream_t st, double* gsum) {
    k_group_finalize<T><<<dim3((unsigned)((d + kBlock - 1) / kBlock), c), kBlock, 0, st>>>(
        partial, d, counts, seg_first, C, gsum);
}

int64_t changed_sort_scratch_ints(int64_t n, int c) {
    return ((n + kSortChunk - 1) / kSortChunk) * (int64_t)(2 * c);
}

int changed_max_segments(int64_t moved, int c) {
    const int64_t entries = 2 * moved;
    return (int)((entries + kSegCols - 1) / kSegCols + std::min<int64_t>(2 * (int64_t)c, entries));
}

void launch_changed_sort(const int32_t* new_labels, const int32_t* old_labels, int64_t n, int c,
                         int32_t* bc, const int32_t* counts_old, int32_t* counts_new, int32_t* perm,
                         int32_t* seg_begin, int32_t* seg_len, int32_t* seg_first, int32_t* nseg,
                         int max_seg, hipStream_t st) {
    const int nb = (int)((n + kSortChunk - 1) / kSortChunk);
    k_chg_hist<<<nb, kSortChunk, 0, st>>>(new_labels, old_labels, (int)n, c, bc);
    k_chg_scan<<<1, kMaxGroups, 0, st>>>(bc, nb, c, counts_old, counts_new, seg_begin, seg_len,
                                         seg_first, nseg, max_seg);
    k_chg_scatter<<<nb, kSortChunk, 0, st>>>(new_labels, old_labels, (int)n, c, bc, perm);
}

template <typename T>
void launch_group_update(const double* partial, int64_t d, int c, const int32_t* counts_new,
                         const int32_t* seg_first, double* gsum, T* C, int32_t* counts_out,
                         hipStream_t st) {
    k_group_update<T><<<dim3((unsigned)((d + kBlock - 1) / kBlock), c), kBlock, 0, st>>>(
        partial, d, c, counts_new, seg_first, gsum, C, counts_out);
}

template <typename T>
void launch_col_sqnorm(const T* C, int64_t d, int c, double* out, hipStream_t st) {
    k_col_sqnorm<T><<<c, kBlock, 0, st>>>(C, d, out);
}

int sweep_seg_partials(int64_t d, int64_t n, int c) { return max_segments(n, c) * row_blocks(d); }

template <typename T>
int launch_sweep_seg(const T* X, int64_t ldx, T* L, int64_t ldl, T* S, int64_t lds, T* Th,
                     int64_t ldt, const T* C, const int32_t* labels, const int32_t* perm,
                     const int32_t* seg_begin, const int32_t* seg_len, const int32_t* nseg,
                     int64_t d, int64_t n, int c, double alpha, double beta, double rho,
                     double inv_rho, double inv_rho_next, double* norm_partial,
                     double* next_partial, hipStream_t st, const double* l21_fac) {
    const int nrb = row_blocks(d);
    const unsigned grid = (unsigned)max_segments(n, c) * (unsigned)nrb;
    constexpr int VV = 16 / sizeof(T);
    const int v = pick_vec<T>(d, {{X, ldx}, {L, ldl}, {S, lds}, {Th, ldt}, {C, d}});
    auto go = [&](auto kern) {
        kern<<<grid, kBlock, 0, st>>>(X, ldx, L, ldl, S, lds, Th, ldt, C, labels, perm, seg_begin,
                                      seg_len, nseg, d, nrb, (T)alpha, (T)beta, (T)rho,
                                      (T)inv_rho, (T)inv_rho_next, norm_partial, next_partial,
                                      l21_fac, T(0), T(0));
    };
    const bool nt = stream_nt<T>(d, n);
    if (l21_fac) {
        if (v == VV) nt ? go(k_sweep_seg<T, VV, true, false, 4, true>) : go(k_sweep_seg<T, VV, true>);
        else nt ? go(k_sweep_seg<T, 1, true, false, 4, true>) : go(k_sweep_seg<T, 1, true>);
    } else {
        if (v == VV) nt ? go(k_sweep_seg<T, VV, false, false, 4, true>) : go(k_sweep_seg<T, VV, false>);
        else nt ? go(k_sweep_seg<T, 1, false, false, 4, true>) : go(k_sweep_seg<T, 1, false>);
    }
    return (int)grid;
}

template <typename T>
int launch_sweep_seg_compact(const T* X, int64_t ldx, T* L, int64_t ldl, T* B, int64_t ldb,
                             const T* C, const int32_t* labels, const int32_t* perm,
                             const int32_t* seg_begin, const int32_t* seg_len, const int32_t* nseg,
                             int64_t d, int64_t n, int c, double alpha, double beta, double rho,
                             double inv_rho, double inv_rho_next, double rho_prev,
                             double inv_rho_prev, double* norm_partial, double* next_partial,
                             hipStream_t st) {
    const int nrb = row_blocks(d);
    const unsigned grid = (unsigned)max_segments(n, c) * (unsigned)nrb;
    constexpr int VV = 16 / sizeof(T);
    const int v = pick_vec<T>(d, {{X, ldx}, {L, ldl}, {B, ldb}, {C, d}});
    auto go = [&](auto kern) {
        kern<<<grid, kBlock, 0, st>>>(X, ldx, L, ldl, B, ldb, nullptr, 0, C, labels, perm, seg_begin,
                                      seg_len, nseg, d, nrb, (T)alpha, (T)beta, (T)rho,
                                      (T)inv_rho, (T)inv_rho_next, norm_partial, next_partial,
                                      nullptr, (T)rho_prev, (T)inv_rho_prev);
    };
    // eight columns in flight per thread (2, 4, 6, 8 measured: 8 is the fastest
    // at 10^4 x 10^4 despite two waves per SIMD)
    // large arrays nontemporal (see stream_nt)
    const bool nt = stream_nt<T>(d, n);
    if (v == VV) nt ? go(k_sweep_seg<T, VV, false, true, 8, true>) : go(k_sweep_seg<T, VV, false, true, 8>);
    else nt ? go(k_sweep_seg<T, 1, false, true, 8, true>) : go(k_sweep_seg<T, 1, false, true, 8>);
    return (int)grid;
}

template <typename T>
void launch_group_partial_compact(const T* X, int64_t ldx, const T* B, int64_t ldb, T inv_rho,
                                  T rho_prev, T inv_rho_prev, int64_t d, int64_t n, int c,
                                  const int32_t* perm, const int32_t* seg_begin,
                                  const int32_t* seg_len, const int32_t* nseg, double* partial,
                                  hipStream_t st) {
    const int nrb = row_blocks(d);
    const unsigned grid = (unsigned)max_segments(n, c) * (unsigned)nrb;
    if (grid == 0) return;
    constexpr int VV = 16 / sizeof(T);
    const int v = pick_vec<T>(d, {{X, ldx}, {B, ldb}});
    auto go = [&](auto kern) {
        kern<<<grid, kBlock, 0, st>>>(X, ldx, B, ldb, nullptr, 0, inv_rho, d, perm, seg_begin,
                                      seg_len, nseg, nrb, partial, rho_prev, inv_rho_prev);
    };
    const bool nt = stream_nt<T>(d, n);
    if (v == VV) nt ? go(k_group_partial<T, VV, true, true, true>) : go(k_group_partial<T, VV, true, true>);
    else nt ? go(k_group_partial<T, 1, true, true, true>) : go(k_group_partial<T, 1, true, true>);
}

// S = soft(B, tau) in place over a d x n column-major matrix.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_soft_inplace(T* __restrict__ B, int64_t ldb, int64_t d,
                                                         int64_t n, T tau) {
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < d;
             i += (int64_t)gridDim.x * kBlock)
            B[j * ldb + i] = soft_threshold(B[j * ldb + i], tau);
}

template <typename T>
void launch_soft_inplace(T* B, int64_t ldb, int64_t d, int64_t n, double tau, hipStream_t st) {
    if (d == 0 || n == 0) return;
    const int64_t bx = (d + kBlock - 1) / kBlock;
    const int64_t by = n < 16384 ? n : 16384;   // columns strided beyond that
    k_soft_inplace<T><<<dim3((unsigned)(bx < 64 ? bx : 64), (unsigned)by), kBlock, 0, st>>>(B, ldb, d, n,
                                                                                         (T)tau);
}

template <typename T>
void launch_l21_factor(const T* X, int64_t ldx, const T* S, int64_t lds, const T* Th, int64_t ldt,
                       const T* C, const int32_t* labels, int64_t d, int64_t n, double alpha,
                       double beta, double rho, double inv_rho, double* fac, hipStream_t st) {
    constexpr int VV = 16 / sizeof(T);
    const int v = pick_vec<T>(d, {{X, ldx}, {S, lds}, {Th, ldt}, {C, d}});
    const unsigned grid = (unsigned)(n < 65536 ? n : 65536);
    auto go = [&](auto kern) {
        kern<<<grid, kBlock, 0, st>>>(X, ldx, S, lds, Th, ldt, C, labels, d, n, (T)alpha, (T)beta,
                                      (T)inv_rho, rho, fac);
    };
    const bool nt = stream_nt<T>(d, n);
    if (v == VV) nt ? go(k_l21_factor<T, VV, true>) : go(k_l21_factor<T, VV>);
    else nt ? go(k_l21_factor<T, 1, true>) : go(k_l21_factor<T, 1>);
}

int64_t dots_slice_rows(int64_t d, int64_t n, int c) {
    const int64_t ct = c <= 32 ? 32 : (c <= 64 ? 64 : 128);
    const int64_t tiles = ((n + 63) / 64) * ((c + ct - 1) / ct);
    int64_t slices = (512 + tiles - 1) / tiles;                 // about 512 workgroups
    const int64_t stages = (d + 31) / 32;
    if (slices > stages) slices = stages;
    if (slices < 1) slices = 1;
    int64_t rows = ((d + slices - 1) / slices + 31) / 32 * 32;  // whole 32-row stages
    if (rows > kRowsPerBlock) rows = kRowsPerBlock;
    return rows;
}

int dots_slices(int64_t d, int64_t n, int c) {
    const int64_t rows = dots_slice_rows(d, n, c);
    return (int)((d + rows - 1) / rows);
}

template <typename T>
void launch_dots(const T* C, int64_t d, int c, const T* Y, int64_t ldy, int64_t n, T* part,
                 hipStream_t st) {
    const int64_t rows = dots_slice_rows(d, n, c);
    const unsigned gx = (unsigned)((n + 63) / 64), gz = (unsigned)dots_slices(d, n, c);
    if (c <= 32)
        k_dots<T, 2><<<dim3(gx, (c + 31) / 32, gz), kBlock, 0, st>>>(C, d, c, Y, ldy, n, rows, part);
    else if (c <= 64)
        k_dots<T, 4><<<dim3(gx, (c + 63) / 64, gz), kBlock, 0, st>>>(C, d, c, Y, ldy, n, rows, part);
    else
        k_dots<T, 8><<<dim3(gx, (c + 127) / 128, gz), kBlock, 0, st>>>(C, d, c, Y, ldy, n, rows, part);
}

template <typename T>
int launch_argmin(const T* part, int nrb, int c, int64_t n, const double* cnorm,
                  const int32_t* old_labels, int32_t* new_labels, double* changed_partial,
                  hipStream_t st) {
    const int g = (int)((n + 15) / 16);
    k_argmin<T><<<g, kBlock, 0, st>>>(part, nrb, c, n, cnorm, old_labels, new_labels,
                                      changed_partial);
    return g;
}

template <typename T>
void launch_d2(const T* Y, int64_t ldy, int64_t d, int64_t n, const int32_t* seeds, int m,
               double* d2, hipStream_t st) {
    const int per = kBlock / 64;
    const unsigned g = (unsigned)((n + per - 1) / per);
    constexpr int VV = 16 / sizeof(T);
    if (pick_vec<T>(d, {{Y, ldy}}) == VV)
        k_d2<T, VV><<<g, kBlock, 0, st>>>(Y, ldy, d, n, seeds, m, d2);
    else
        k_d2<T, 1><<<g, kBlock, 0, st>>>(Y, ldy, d, n, seeds, m, d2);
}

int64_t d2_copy_ld(int64_t d) { return (d + 7) / 8 * 8; }

void launch_d2_first(const float* Y, int64_t ldy, int64_t d, int64_t n, const int32_t* seeds,
                     double* d2, _Float16* Z, float* zsc, double* ynorm, hipStream_t st) {
    const int per = kBlock / 64;
    const unsigned g = (unsigned)((n + per - 1) / per);
    const int64_t ldz = d2_copy_ld(d);
    if (pick_vec<float>(d, {{Y, ldy}}) == 4)
        k_d2_first<4><<<g, kBlock, 0, st>>>(Y, ldy, d, n, seeds, d2, Z, ldz, zsc, ynorm);
    else
        k_d2_first<1><<<g, kBlock, 0, st>>>(Y, ldy, d, n, seeds, d2, Z, ldz, zsc, ynorm);
}

void launch_d2_bounded(const float* Y, int64_t ldy, int64_t d, int64_t n, const int32_t* seeds,
                       int m, double* d2, const _Float16* Z, const float* zsc, const double* ynorm,
                       hipStream_t st) {
    const int per = kBlock / 64;
    const unsigned g = (unsigned)((n + per - 1) / per);
    // FP32 error of A: per-term rounding (3 units) plus at most 8 ceil(d / 512) lane
    // additions, doubled
    const float eta = (float)(2.0 * (3.0 + 8.0 * (double)((d + 511) / 512)) * std::ldexp(1.0, -24));
    // (the FP16 copy, 2 d n bytes, is re-read by every seed's pass: plain loads,
    // which keep part of it in the last-level cache; nontemporal ones cost 4.7 ->
    // 5.5 ms of seeding per 10^4 x 10^4 solve)
    if (pick_vec<float>(d, {{Y, ldy}}) == 4)
        k_d2_bounded<4><<<g, kBlock, 0, st>>>(Y, ldy, d, n, seeds, m, d2, Z, d2_copy_ld(d), zsc,
                                              ynorm, eta);
    else
        k_d2_bounded<1><<<g, kBlock, 0, st>>>(Y, ldy, d, n, seeds, m, d2, Z, d2_copy_ld(d), zsc,
                                              ynorm, eta);
}

void launch_pick(const double* d2, int64_t n, const double* u, int m, int32_t* seeds,
                 int32_t* chosen, hipStream_t st) {
    k_pick<<<1, kPickThreads, 0, st>>>(d2, n, u, m, seeds, chosen);
}

template <typename T>
void launch_gather_cols(const T* Y, int64_t ldy, int64_t d, const int32_t* idx, int c, T* C,
                        hipStream_t st) {
    k_gather_cols<T><<<dim3((unsigned)((d + kBlock - 1) / kBlock), c), kBlock, 0, st>>>(Y, ldy, d,
                                                                                          idx, C);
}

// ------------------------------------------------------ instantiations

#define RESPCA_INSTANTIATE(T)                                                                      \
    template void launch_zero2d<T>(T*, int64_t, int64_t, int64_t, hipStream_t);                    \
    template int launch_sumsq<T>(const T*, int64_t, int64_t, int64_t, double*, hipStream_t);       \
    template void launch_group_partial<T>(bool, const T*, int64_t, const T*, int64_t, const T*,     \
                                          int64_t, T, int64_t, int64_t, int, const int32_t*,       \
                                          const int32_t*, const int32_t*, const int32_t*, double*, \
                                          hipStream_t, int);                                       \
    template void launch_group_finalize<T>(const double*, int64_t, int, const int32_t*,            \
                                           const int32_t*, T*, hipStream_t, double*);              \
    template void launch_group_update<T>(const double*, int64_t, int, const int32_t*,              \
                                         const int32_t*, double*, T*, int32_t*, hipStream_t);      \
    template void launch_col_sqnorm<T>(const T*, int64_t, int, double*, hipStream_t);              \
    template int launch_sweep_seg<T>(const T*, int64_t, T*, int64_t, T*, int64_t, T*, int64_t,    \
                                     const T*, const int32_t*, const int32_t*, const int32_t*,     \
                                     const int32_t*, const int32_t*, int64_t, int64_t, int,        \
                                     double, double, double, double, double, double*, double*,     \
                                     hipStream_t, const double*);                                  \
    template int launch_sweep_seg_compact<T>(const T*, int64_t, T*, int64_t, T*, int64_t,         \
                                             const T*, const int32_t*, const int32_t*,             \
                                             const int32_t*, const int32_t*, const int32_t*,       \
                                             int64_t, int64_t, int, double, double, double,        \
                                             double, double, double, double, double*, double*,     \
                                             hipStream_t);                                         \
    template void launch_group_partial_compact<T>(const T*, int64_t, const T*, int64_t, T, T, T,  \
                                                  int64_t, int64_t, int, const int32_t*,           \
                                                  const int32_t*, const int32_t*, const int32_t*,  \
                                                  double*, hipStream_t);                           \
    template void launch_soft_inplace<T>(T*, int64_t, int64_t, int64_t, double, hipStream_t);     \
    template void launch_l21_factor<T>(const T*, int64_t, const T*, int64_t, const T*, int64_t,   \
                                       const T*, const int32_t*, int64_t, int64_t, double, double,  \
                                       double, double, double*, hipStream_t);                      \
    template void launch_dots<T>(const T*, int64_t, int, const T*, int64_t, int64_t, T*,           \
                                 hipStream_t);                                                     \
    template int launch_argmin<T>(const T*, int, int, int64_t, const double*, const int32_t*,     \
                                  int32_t*, double*, hipStream_t);                                 \
    template void launch_d2<T>(const T*, int64_t, int64_t, int64_t, const int32_t*, int, double*, \
                               hipStream_t);                                                       \
    template void launch_gather_cols<T>(const T*, int64_t, int64_t, const int32_t*, int, T*,      \
                                        hipStream_t);

RESPCA_INSTANTIATE(float)
RESPCA_INSTANTIATE(double)

}  // namespace respca
