// Host runtime and C ABI of librespca: handle/workspace management, argument
// checks, and the RES-PCA driver loop (initial K-means, then outer ALM
// iterations L -> p -> S -> Theta/rho until the Sec. 5 criterion holds).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/respca.h"
#include "handle.h"
#include "kernels.h"
#include "spectral.h"

using namespace respca;

// Workspace of respca_iterate_noalloc: a fixed device array, one copy per GPU,
// held until the process ends.  Host code never passes this name to a kernel
// (on the host it is only a stand-in for the symbol); it uses the per-device
// address that respca_create looks up with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[RESPCA_NOALLOC_SCRATCH_BYTES];

namespace {

const char* kVersion = "librespca 0.3 (gfx950)";

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device (= `device`), looked up
// once per device.
respca_status lookup_scratch(respca_handle h, int device) {
    if (device >= kMaxScratchDevices) return RESPCA_OK;   // the no-alloc call reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return RESPCA_OK;
    void* ptr = nullptr;
    CK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = (char*)ptr;
    return RESPCA_OK;
}

// Host polling of a readback gives up after this long and synchronizes the stream
// (which also reports a failed kernel).
constexpr double kStatusSpinSeconds = 2e-3;

// Publishes `count` status words to pinned host memory: the words first, then,
// after a system-scope fence, the sequence number the host waits for.  Word 4
// (columns refined by the last assignment pass) is cleared once published, so
// each pass is counted once.  One thread; the stores are ordinary vector stores.
__global__ void k_publish_status(double* __restrict__ words, int count,
                                 volatile double* host_words, volatile uint64_t* host_seq,
                                 uint64_t seq) {
    if (threadIdx.x != 0) return;
    for (int i = 0; i < count; ++i) host_words[i] = words[i];
    if (count > 4) words[4] = 0.0;
    __threadfence_system();
    *host_seq = seq;
    __threadfence_system();
}

// Fold finished event pairs into the counters; call once the work they bracket has
// finished (a pair whose end event still reads as pending is waited for).
void prof_resolve(respca_handle h) {
    for (auto& p : h->prof_pending) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e == hipErrorNotReady && hipEventSynchronize(p.b) == hipSuccess)
            e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e == hipSuccess) {
            h->prof_launches[p.kernel] += 1;
            h->prof_ms[p.kernel] += ms;
            h->prof_bytes[p.kernel] += p.bytes;
            h->prof_flops[p.kernel] += p.flops;
        }
        h->prof_pool.push_back(p.a);
        h->prof_pool.push_back(p.b);
    }
    h->prof_pending.clear();
}

}  // namespace

respca_status respca::resolve(respca_handle h, const respca_params* p, int64_t d, int64_t n, Resolved& r) {
    if (!p) return fail(h, RESPCA_ERR_INVALID, "params is NULL");
    if (d < 1 || n < 1 || d >= (int64_t)INT32_MAX || n >= (int64_t)INT32_MAX)
        return fail(h, RESPCA_ERR_INVALID, "d and n must be in [1, 2^31)");
    r.lambda = std::isnan(p->lambda) ? std::sqrt((double)(d > n ? d : n)) : p->lambda;
    r.c = p->rank == 0 ? 5 : p->rank;
    r.tol = p->tol;
    r.max_iter = p->max_iter;
    r.rho0 = p->rho0;
    r.kappa = p->kappa;
    r.rho_max = p->rho_max;
    r.max_lloyd = p->max_lloyd;
    r.precision = p->precision;
    r.sparse_norm = p->sparse_norm;
    r.pstep = p->pstep;
    r.sigma = p->spectral_sigma;
    r.seed = p->seed;
    r.init_labels = p->init_labels;
    r.history = p->history;
    r.init_embedding = p->init_labels ? nullptr : (const float*)p->init_embedding;
    r.emb_ld = p->init_embedding_ld;
    r.emb_rows = p->init_embedding_rows;
    r.emb_refine = p->init_embedding_refine;
    if (r.init_embedding) {
        if (r.emb_rows < 1 || r.emb_ld < r.emb_rows)
            return fail(h, RESPCA_ERR_INVALID, "init_embedding rows/leading dimension invalid");
        if (p->precision == RESPCA_F64)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "init_embedding needs an FP32 precision");
        if (r.emb_refine < 0 || r.emb_refine > 2)
            return fail(h, RESPCA_ERR_INVALID, "init_embedding_refine must be 0, 1 or 2");
    }
    if (!(r.lambda >= 0.0) || !std::isfinite(2.0 * r.lambda))
        return fail(h, RESPCA_ERR_INVALID, "lambda must be finite and >= 0");
    if (r.c < 1 || (int64_t)r.c > n) return fail(h, RESPCA_ERR_INVALID, "rank must be in [1, n]");
    if (r.c > kMaxGroups) return fail(h, RESPCA_ERR_UNSUPPORTED, "rank above 1024 is not supported");
    if (!(r.tol >= 0.0)) return fail(h, RESPCA_ERR_INVALID, "tol must be >= 0");
    if (r.sparse_norm != RESPCA_SPARSE_L1 && r.sparse_norm != RESPCA_SPARSE_L21)
        return fail(h, RESPCA_ERR_INVALID, "sparse_norm must be RESPCA_SPARSE_L1 or RESPCA_SPARSE_L21");
    if (r.max_iter < 1) return fail(h, RESPCA_ERR_INVALID, "max_iter must be >= 1");
    if (!(r.rho0 > 0.0) || !std::isfinite(r.rho0)) return fail(h, RESPCA_ERR_INVALID, "rho0 must be > 0");
    if (!(r.kappa > 1.0) || !std::isfinite(r.kappa)) return fail(h, RESPCA_ERR_INVALID, "kappa must be > 1");
    if (!(r.rho_max >= r.rho0)) return fail(h, RESPCA_ERR_INVALID, "rho_max must be >= rho0");
    if (r.max_lloyd < 1) return fail(h, RESPCA_ERR_INVALID, "max_lloyd must be >= 1");
    if (r.precision != RESPCA_F64 && r.precision != RESPCA_F32 && r.precision != RESPCA_BF16GEMM_F32)
        return fail(h, RESPCA_ERR_INVALID, "unknown precision");
    if (r.pstep != RESPCA_PSTEP_KMEANS && r.pstep != RESPCA_PSTEP_SPECTRAL)
        return fail(h, RESPCA_ERR_INVALID, "pstep must be RESPCA_PSTEP_KMEANS or RESPCA_PSTEP_SPECTRAL");
    if (r.pstep == RESPCA_PSTEP_SPECTRAL) {
        if (r.sigma == 0.0 || !std::isfinite(r.sigma))
            return fail(h, RESPCA_ERR_INVALID, "spectral_sigma must be finite and nonzero");
        if (r.c > kSpectralMaxGroups || n > kSpectralMaxN)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "spectral p-step: c <= 40 and n <= 32768");
        if (r.init_embedding)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "spectral p-step: no init_embedding");
    }
    return RESPCA_OK;
}

namespace {

struct Span {
    uintptr_t lo, hi;
};

Span span_of(const void* p, int64_t ld, int64_t d, int64_t n, size_t w) {
    uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return {lo, lo + (uintptr_t)((ld * (n - 1) + d) * (int64_t)w)};
}

bool overlap(Span a, Span b) { return a.lo < b.hi && b.lo < a.hi; }

// ------------------------------------------------------------------- engine

template <typename T>
struct Engine {
    respca_handle h;
    hipStream_t st;
    int64_t d, n;
    int c;
    bool bf16;       // split-bf16 MFMA distances with exact refinement (float runs)
    int nrb;
    double* status;  // device words: [0..2] norms^2, [3] changed count, [4] refined columns
    int64_t refined = 0;
    uint64_t published_seq = 0;   // sequence number of words already being published
    bool next_ready = false;   // pmeans / sort tables hold the next L-step's group sums of D

    respca_status setup() {
        nrb = row_blocks(d);
        const size_t segs = (size_t)max_segments(n, c);
        CKS(ensure(h, h->perm, n * sizeof(int32_t)));
        CKS(ensure(h, h->counts, c * sizeof(int32_t)));
        CKS(ensure(h, h->segb, segs * sizeof(int32_t)));
        CKS(ensure(h, h->segl, segs * sizeof(int32_t)));
        CKS(ensure(h, h->segf, (c + 1) * sizeof(int32_t)));
        CKS(ensure(h, h->nseg, sizeof(int32_t)));
        CKS(ensure(h, h->pmeans, segs * d * sizeof(double)));
        CKS(ensure(h, h->sortbc, (size_t)sort_scratch_ints(n, c) * sizeof(int32_t)));
        CKS(ensure(h, h->dots, assign_workspace_bytes<T>(d, n, c)));
        CKS(ensure(h, h->cnorm, c * sizeof(double)));
        CKS(ensure(h, h->lab_a, n * sizeof(int32_t)));
        CKS(ensure(h, h->lab_b, n * sizeof(int32_t)));
        size_t np = (size_t)sweep_seg_partials(d, n, c);
        const size_t nsum = (size_t)nrb * (size_t)((n + 15) / 16);
        if (nsum > np) np = nsum;
        CKS(ensure(h, h->normp, 3 * np * sizeof(double)));
        CKS(ensure(h, h->chgp, (size_t)assign_partials_max(n) * sizeof(double)));
        // status words in device memory (in the scratch area while arena_on);
        // readback() brings them to the host
        CKS(ensure(h, h->status, 8 * sizeof(double)));
        status = (double*)h->status.p;
        if (h->arena_on) return RESPCA_OK;
        CK(hipMemsetAsync(status, 0, 8 * sizeof(double), st));
        CKS(ensure_host(h, (16 + 2 * (size_t)c) * sizeof(double)));
        if (!h->hstatus) {   // pinned host copy: words 0..7, sequence number in word 8
            CK(hipHostMalloc((void**)&h->hstatus, 16 * sizeof(double), hipHostMallocMapped));
            CK(hipHostGetDevicePointer((void**)&h->hstatus_dev, h->hstatus, 0));
            std::memset(h->hstatus, 0, 16 * sizeof(double));
            h->status_seq = 0;
        }
        return RESPCA_OK;
    }

    // Every buffer respca_iterate's steps use (setup, Lloyd's group sums and
    // moved-column update, the l2,1 factors), at their largest sizes.
    respca_status reserve_iterate(const Resolved& r) {
        CKS(setup());
        double* gs = nullptr;
        CKS(group_sums(gs));
        CKS(reserve_update());
        if (r.sparse_norm == RESPCA_SPARSE_L21) CKS(ensure(h, h->l21f, (size_t)n * sizeof(double)));
        return RESPCA_OK;
    }

    int32_t* perm() { return (int32_t*)h->perm.p; }
    int32_t* counts() { return (int32_t*)h->counts.p; }

    respca_status readback(double out[4]) {
        CK(hipGetLastError());
        if (h->arena_on) {
            double w[5];
            CK(hipMemcpyAsync(w, status, sizeof(w), hipMemcpyDeviceToHost, st));
            CK(hipStreamSynchronize(st));
            for (int i = 0; i < 4; ++i) out[i] = w[i];
            refined += (int64_t)w[4];
            return RESPCA_OK;
        }
        // The words reach the host behind a sequence number; polling it costs a few
        // microseconds where a stream synchronization costs ~20 (a pass is a chain
        // of short kernels, so this is paid every Lloyd pass and every iteration).
        uint64_t seq = published_seq;   // set when the last kernel published the words
        published_seq = 0;
        if (seq == 0) {
            seq = ++h->status_seq;
            k_publish_status<<<1, 64, 0, st>>>(status, 5, h->hstatus_dev,
                                               (uint64_t*)(h->hstatus_dev + 8), seq);
            CK(hipGetLastError());
        }
        volatile uint64_t* hseq = (volatile uint64_t*)(h->hstatus + 8);
        {
            const auto t0 = std::chrono::steady_clock::now();
            while (*hseq != seq &&
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() <
                       kStatusSpinSeconds) {
            }
        }
        if (*hseq != seq) {
            CK(hipStreamSynchronize(st));
            if (*hseq != seq) return fail(h, RESPCA_ERR_HIP, "status words did not reach the host");
        }
        const volatile double* w = h->hstatus;
        for (int i = 0; i < 4; ++i) out[i] = w[i];
        refined += (int64_t)w[4];
        prof_resolve(h);
        return RESPCA_OK;
    }

    respca_status sumsq(const T* X, int64_t ldx, double& out) {
        const int np = launch_sumsq<T>(X, ldx, d, n, (double*)h->normp.p, st);
        launch_sum_partials((double*)h->normp.p, np, 1, status, st);
        double s[4];
        CKS(readback(s));
        out = s[0];
        return RESPCA_OK;
    }

    void sort(const int32_t* labels) {
        launch_label_sort(labels, n, c, (int32_t*)h->sortbc.p, counts(), perm(), (int32_t*)h->segb.p,
                          (int32_t*)h->segl.p, (int32_t*)h->segf.p, (int32_t*)h->nseg.p, st);
    }

    // C[:, k] <- mean over group k of Y (Y = X - S + Theta*inv_rho when with_d),
    // for the groups of the last sort; empty groups keep C[:, k].  With gsum the
    // group sums (double) are kept for incremental updates.
    void group_means(bool with_d, const T* A, int64_t lda, const T* S, int64_t lds, const T* Th,
                     int64_t ldt, T inv_rho, T* C, double* gsum = nullptr) {
        {
            ProfScope ps(h, st, RESPCA_KERNEL_MEANS, (with_d ? 3.0 : 1.0) * (double)d * n * sizeof(T));
            launch_group_partial<T>(with_d, A, lda, S, lds, Th, ldt, inv_rho, d, n, c, perm(),
                                (const int32_t*)h->segb.p, (const int32_t*)h->segl.p,
                                (const int32_t*)h->nseg.p, (double*)h->pmeans.p, st);
        }
        launch_group_finalize<T>((const double*)h->pmeans.p, d, c, counts(),
                                 (const int32_t*)h->segf.p, C, st, gsum);
    }

    // Columns an assignment pass may move for the incremental means (more: a
    // full means pass).
    int64_t moved_cap() const { return n / 8; }

    // Group sums (double, d x c) kept by the full means passes of Lloyd.
    respca_status group_sums(double*& out) {
        CKS(ensure(h, h->gsum, (size_t)c * d * sizeof(double)));
        out = (double*)h->gsum.p;
        return RESPCA_OK;
    }

    // C and the group sums for labels `neu` from those for labels `old`, moving
    // only the `moved` columns whose label changed (moved <= moved_cap()); the
    // group counts follow.  The sort tables are left as they were (the caller
    // re-sorts before it needs them).
    respca_status reserve_update() {
        const int maxs = changed_max_segments(moved_cap(), c);
        CKS(ensure(h, h->cnt2, c * sizeof(int32_t)));
        CKS(ensure(h, h->cbc, (size_t)changed_sort_scratch_ints(n, c) * sizeof(int32_t)));
        CKS(ensure(h, h->cperm, 2 * (size_t)n * sizeof(int32_t)));
        CKS(ensure(h, h->csegb, (size_t)maxs * sizeof(int32_t)));
        CKS(ensure(h, h->csegl, (size_t)maxs * sizeof(int32_t)));
        CKS(ensure(h, h->csegf, (2 * (size_t)c + 1) * sizeof(int32_t)));
        CKS(ensure(h, h->cnseg, sizeof(int32_t)));
        CKS(ensure(h, h->cpart, (size_t)maxs * d * sizeof(double)));
        return RESPCA_OK;
    }

    respca_status update_means(const T* Y, int64_t ldy, const int32_t* neu, const int32_t* old,
                               int64_t moved, T* C) {
        const int maxs = changed_max_segments(moved_cap(), c);
        CKS(reserve_update());
        int32_t* cnt2 = (int32_t*)h->cnt2.p;
        launch_changed_sort(neu, old, n, c, (int32_t*)h->cbc.p, counts(), cnt2, (int32_t*)h->cperm.p,
                            (int32_t*)h->csegb.p, (int32_t*)h->csegl.p, (int32_t*)h->csegf.p,
                            (int32_t*)h->cnseg.p, maxs, st);
        {
            ProfScope ps(h, st, RESPCA_KERNEL_MEANS, 2.0 * (double)moved * d * sizeof(T));
            launch_group_partial<T>(false, Y, ldy, nullptr, 0, nullptr, 0, T(0), d, n, c,
                                    (const int32_t*)h->cperm.p, (const int32_t*)h->csegb.p,
                                    (const int32_t*)h->csegl.p, (const int32_t*)h->cnseg.p,
                                    (double*)h->cpart.p, st, changed_max_segments(moved, c));
        }
        launch_group_update<T>((const double*)h->cpart.p, d, c, cnt2, (const int32_t*)h->csegf.p,
                               (double*)h->gsum.p, C, counts(), st);
        return RESPCA_OK;
    }

    // Assignment pass: new = nearest centroid of every column of Y; status[3] = #changed.
    void assign(const T* Y, int64_t ldy, const T* C, const int32_t* old, int32_t* neu) {
        if (!bf16) launch_col_sqnorm<T>(C, d, c, (double*)h->cnorm.p, st);   // bf16: in the pass
        int g = 0, extra = 0;
        {
            ProfScope ps(h, st, RESPCA_KERNEL_DISTANCE, (double)d * n * sizeof(T),
                         2.0 * (double)c * (double)d * (double)n);
            g = launch_assign<T>(C, d, c, Y, ldy, n, (double*)h->cnorm.p, old, neu, h->dots.p,
                                 (double*)h->chgp.p, bf16, &extra, st);
        }
        // the finishing kernel also publishes the words for the readback that follows
        StatusPublish pub;
        if (!h->arena_on) {
            pub.words = status;
            pub.host = h->hstatus_dev;
            pub.host_seq = (uint64_t*)(h->hstatus_dev + 8);
            pub.seq = ++h->status_seq;
            published_seq = pub.seq;
        }
        launch_assign_finish((const double*)h->chgp.p, g,
                             extra ? assign_refine_counters(h->dots.p, d, n, c) : nullptr, status + 3,
                             st, pub);
    }

    // Lloyd passes on the columns of Y from (cur, C); see oracle_lloyd for the
    // exact rule.  `first` receives the status of the first pass.  sums_valid:
    // the group sums hold those of Y for the labels in cur (left by the caller's
    // means pass); then, and after each full means pass here, a pass that moved
    // few columns updates the means from the moved columns only.
    respca_status lloyd(const T* Y, int64_t ldy, T* C, int32_t*& cur, int32_t*& alt, int max_lloyd,
                        int& steps, double first[4], bool sums_valid = false) {
        steps = 0;
        bool have = sums_valid;
        while (steps < max_lloyd) {
            assign(Y, ldy, C, cur, alt);
            double s[4];
            CKS(readback(s));
            if (steps == 0 && first) std::memcpy(first, s, sizeof(s));
            ++steps;
            if (s[3] == 0.0) break;
            std::swap(cur, alt);
            const int64_t moved = (int64_t)s[3];
            if (have && moved <= moved_cap()) {
                CKS(update_means(Y, ldy, cur, alt, moved, C));
            } else {
                double* gs = nullptr;
                CKS(group_sums(gs));
                sort(cur);
                group_means(false, Y, ldy, nullptr, 0, nullptr, 0, T(0), C, gs);
                have = true;
            }
        }
        return RESPCA_OK;
    }

    // K-means of the columns of Y: k-means++ seeds, nearest-seed groups, their
    // means (empty groups keep the seed), then Lloyd.
    respca_status kmeans(const T* Y, int64_t ldy, uint64_t seed, int max_lloyd, T* C,
                         int32_t*& cur, int32_t*& alt, int& steps) {
        CKS(place_seeds(Y, ldy, seed));
        return from_seeds(Y, ldy, max_lloyd, C, cur, alt, steps);
    }

    // k-means++ seeding of the columns of Y (splitmix64(seed) uniforms): the c seed
    // column indices in h->seeds.
    respca_status place_seeds(const T* Y, int64_t ldy, uint64_t seed) {
        CKS(ensure(h, h->d2, n * sizeof(double)));
        CKS(ensure(h, h->chosen, n * sizeof(int32_t)));
        CKS(ensure(h, h->seeds, c * sizeof(int32_t)));
        CKS(ensure(h, h->u, c * sizeof(double)));
        uint64_t state = seed;
        double* hu = h->hstage + 8;
        for (int m = 0; m < c; ++m) hu[m] = uniform01(state);
        int64_t s0 = (int64_t)std::floor(hu[0] * (double)n);
        if (s0 >= n) s0 = n - 1;
        int32_t* seeds = (int32_t*)h->seeds.p;
        int32_t* chosen = (int32_t*)h->chosen.p;
        int32_t* hi = (int32_t*)(h->hstage + 4);
        hi[0] = (int32_t)s0;
        hi[1] = 1;
        CK(hipMemcpyAsync(h->u.p, hu, c * sizeof(double), hipMemcpyHostToDevice, st));
        launch_zero_i32(chosen, n, st);
        CK(hipMemcpyAsync(seeds, &hi[0], sizeof(int32_t), hipMemcpyHostToDevice, st));
        CK(hipMemcpyAsync(chosen + s0, &hi[1], sizeof(int32_t), hipMemcpyHostToDevice, st));
        const double pass_bytes = (double)d * n * sizeof(T);
        // float runs with more than 8 seeds: bounded passes over an fp16 copy of Y
        // (same D^2 values; the copy costs one extra pass, so few seeds skip it).
        // Without memory for the copy the plain passes run.
        bool bounded = false;
        if constexpr (std::is_same<T, float>::value) {
            if (c > 8) {
                bounded = ensure(h, h->zcopy, (size_t)d2_copy_ld(d) * n * sizeof(_Float16)) == RESPCA_OK;
                if (!bounded) {
                    (void)hipGetLastError();
                    h->err.clear();
                }
            }
        }
        if (bounded) {
            CKS(ensure(h, h->zsc, n * sizeof(float)));
            CKS(ensure(h, h->ynorm, n * sizeof(double)));
            {
                ProfScope ps(h, st, RESPCA_KERNEL_SEEDING, pass_bytes + (double)d * n * sizeof(_Float16));
                launch_d2_first((const float*)Y, ldy, d, n, seeds, (double*)h->d2.p,
                                (_Float16*)h->zcopy.p, (float*)h->zsc.p, (double*)h->ynorm.p, st);
            }
            for (int m = 1; m < c; ++m) {
                launch_pick((const double*)h->d2.p, n, (const double*)h->u.p, m, seeds, chosen, st);
                ProfScope ps(h, st, RESPCA_KERNEL_SEEDING, (double)d * n * sizeof(_Float16));
                launch_d2_bounded((const float*)Y, ldy, d, n, seeds, m, (double*)h->d2.p,
                                  (const _Float16*)h->zcopy.p, (const float*)h->zsc.p,
                                  (const double*)h->ynorm.p, st);
            }
        } else {
            {
                ProfScope ps(h, st, RESPCA_KERNEL_SEEDING, pass_bytes);
                launch_d2<T>(Y, ldy, d, n, seeds, 0, (double*)h->d2.p, st);
            }
            for (int m = 1; m < c; ++m) {
                launch_pick((const double*)h->d2.p, n, (const double*)h->u.p, m, seeds, chosen, st);
                ProfScope ps(h, st, RESPCA_KERNEL_SEEDING, pass_bytes);
                launch_d2<T>(Y, ldy, d, n, seeds, m, (double*)h->d2.p, st);
            }
        }
        return RESPCA_OK;
    }

    // K-means of the columns of Y from the seeds in h->seeds: centroids = the seed
    // columns of Y, nearest-seed assignment, then Lloyd.
    respca_status from_seeds(const T* Y, int64_t ldy, int max_lloyd, T* C, int32_t*& cur,
                             int32_t*& alt, int& steps) {
        launch_gather_cols<T>(Y, ldy, d, (const int32_t*)h->seeds.p, c, C, st);
        launch_zero_i32(cur, n, st);
        assign(Y, ldy, C, cur, alt);
        std::swap(cur, alt);
        double* gs = nullptr;
        CKS(group_sums(gs));
        sort(cur);
        group_means(false, Y, ldy, nullptr, 0, nullptr, 0, T(0), C, gs);
        CKS(lloyd(Y, ldy, C, cur, alt, max_lloyd, steps, nullptr, true));  // also waits for the pinned stage
        return RESPCA_OK;
    }

    SpectralStats spec;

    // Groups from the row embedding of the columns of Y (spectral clustering):
    // with `fresh`, k-means++ from seed then Lloyd (the initialisation);
    // otherwise Lloyd from the current groups, their centroids the group means of
    // the rows (an empty group at zero).  The K-means runs on a second engine over
    // the c x n embedding, which shares the handle's sort and distance buffers, so
    // the caller's sort tables are stale afterwards.
    respca_status spectral_groups(const Resolved& r, const T* Y, int64_t ldy, bool fresh,
                                  int32_t*& cur, int32_t*& alt, int& steps) {
        CKS(ensure(h, h->sp_emb, (size_t)c * n * sizeof(double)));
        CKS(ensure(h, h->sp_cent, (size_t)c * c * sizeof(double)));
        double* emb = (double*)h->sp_emb.p;
        double* cent = (double*)h->sp_cent.p;
        // after the first embedding of this call the previous Ritz vectors seed the next
        CKS(spectral_embed<T>(h, Y, ldy, d, n, c, r.sigma, r.seed, emb, &spec, st, spec.calls > 0));
        Engine<double> e2{h, st, (int64_t)c, n, c, false};
        CKS(e2.setup());
        steps = 0;
        if (fresh) {
            CKS(e2.kmeans(emb, c, r.seed, r.max_lloyd, cent, cur, alt, steps));
        } else {
            launch_zero2d<double>(cent, c, c, c, st);
            e2.sort(cur);
            e2.group_means(false, emb, c, nullptr, 0, nullptr, 0, 0.0, cent);
            CKS(e2.lloyd(emb, c, cent, cur, alt, r.max_lloyd, steps, nullptr));
        }
        CKS(setup());   // this engine's buffers at its own sizes again
        next_ready = false;
        return RESPCA_OK;
    }

    // One outer iteration; norms receives the three Frobenius norms.  rho_prev > 0
    // selects the compact l1 state: S holds B = X - L + Theta/rho_prev of the
    // previous iteration (S and Theta follow from it) and Th is not used.
    respca_status iterate_once(const Resolved& r, const T* X, int64_t ldx, T* L, int64_t ldl, T* S,
                               int64_t lds, T* Th, int64_t ldt, T* C, int32_t*& cur, int32_t*& alt,
                               double rho, double norms[3], int& steps, double rho_prev = 0.0) {
        const bool compact = rho_prev > 0.0;
        if (compact && r.sparse_norm == RESPCA_SPARSE_L21)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "compact state with the l2,1 penalty");
        const double alpha = rho / (2.0 * r.lambda + rho);
        const double beta = (2.0 * r.lambda) / (2.0 * r.lambda + rho);
        const double inv = 1.0 / rho;
        const double next = r.kappa * rho;                           // Sec. 4.4 schedule
        const double inv_next = 1.0 / (next < r.rho_max ? next : r.rho_max);
        if (next_ready) {
            // the previous sweep summed D over these same groups at this rho
            launch_group_finalize<T>((const double*)h->pmeans.p, d, c, counts(),
                                     (const int32_t*)h->segf.p, C, st);
        } else if (compact) {
            sort(cur);                                               // Sec. 4.1: groups of D
            {
                ProfScope ps(h, st, RESPCA_KERNEL_MEANS, 2.0 * (double)d * n * sizeof(T));
                launch_group_partial_compact<T>(X, ldx, S, lds, (T)inv, (T)rho_prev,
                                                (T)(1.0 / rho_prev), d, n, c, perm(),
                                                (const int32_t*)h->segb.p, (const int32_t*)h->segl.p,
                                                (const int32_t*)h->nseg.p, (double*)h->pmeans.p, st);
            }
            launch_group_finalize<T>((const double*)h->pmeans.p, d, c, counts(),
                                     (const int32_t*)h->segf.p, C, st);
        } else {
            sort(cur);                                               // Sec. 4.1: groups of D
            group_means(true, X, ldx, S, lds, Th, ldt, (T)inv, C);
        }
        const double* fac = nullptr;
        if (r.sparse_norm == RESPCA_SPARSE_L21) {
            // Sec. 3 alternative penalty: the S-step needs ||B_j|| over the whole column
            CKS(ensure(h, h->l21f, (size_t)n * sizeof(double)));
            ProfScope ps(h, st, RESPCA_KERNEL_COLNORM, 3.0 * (double)d * n * sizeof(T));
            launch_l21_factor<T>(X, ldx, S, lds, Th, ldt, C, cur, d, n, alpha, beta, rho, inv,
                                 (double*)h->l21f.p, st);
            fac = (const double*)h->l21f.p;
        }
        int np = 0;
        if (compact) {
            ProfScope ps(h, st, RESPCA_KERNEL_SWEEP, 5.0 * (double)d * n * sizeof(T));
            np = launch_sweep_seg_compact<T>(X, ldx, L, ldl, S, lds, C, cur, perm(),
                                             (const int32_t*)h->segb.p, (const int32_t*)h->segl.p,
                                             (const int32_t*)h->nseg.p, d, n, c, alpha, beta, rho, inv,
                                             inv_next, rho_prev, 1.0 / rho_prev, (double*)h->normp.p,
                                             (double*)h->pmeans.p, st);
        } else {
            ProfScope ps(h, st, RESPCA_KERNEL_SWEEP, 7.0 * (double)d * n * sizeof(T));
            np = launch_sweep_seg<T>(X, ldx, L, ldl, S, lds, Th, ldt, C, cur, perm(),
                                     (const int32_t*)h->segb.p, (const int32_t*)h->segl.p,
                                     (const int32_t*)h->nseg.p, d, n, c, alpha, beta, rho, inv,
                                     inv_next, (double*)h->normp.p, (double*)h->pmeans.p, st, fac);
        }
        launch_sum_partials((const double*)h->normp.p, np, 3, status, st);
        if (r.pstep == RESPCA_PSTEP_SPECTRAL) {
            double s[4];
            CKS(readback(s));   // the sweep's norms, before the p-step reuses the buffers
            for (int i = 0; i < 3; ++i) norms[i] = std::sqrt(s[i]);
            return spectral_groups(r, L, ldl, false, cur, alt, steps);   // Sec. 4.2, nonlinear form
        }
        double first[4];
        CKS(lloyd(L, ldl, C, cur, alt, r.max_lloyd, steps, first));  // Sec. 4.2
        for (int i = 0; i < 3; ++i) norms[i] = std::sqrt(first[i]);
        // unchanged labels: the sort tables and the sweep's sums stay valid
        next_ready = (first[3] == 0.0);
        return RESPCA_OK;
    }
};

template <typename T>
respca_status solve_t(respca_handle h, const Resolved& r, int64_t d, int64_t n, const T* X,
                      int64_t ldx, T* L, int64_t ldl, T* S, int64_t lds, int32_t* labels,
                      respca_info* info, hipStream_t st) {
    Engine<T> e{h, st, d, n, r.c, r.precision == RESPCA_BF16GEMM_F32};
    CKS(e.setup());
    // l1 penalty: the compact state (S holds B = X - L + Theta/rho until the end,
    // when it becomes soft(B, 1/rho)); l2,1: S and Theta as they are
    const bool compact = r.sparse_norm != RESPCA_SPARSE_L21;
    if (!compact) CKS(ensure(h, h->theta, (size_t)d * n * sizeof(T)));
    CKS(ensure(h, h->cbuf, (size_t)d * r.c * sizeof(T)));
    T* Th = compact ? nullptr : (T*)h->theta.p;
    T* C = (T*)h->cbuf.p;
    int32_t* cur = (int32_t*)h->lab_a.p;
    int32_t* alt = (int32_t*)h->lab_b.p;

    double nx2 = 0.0;
    CKS(e.sumsq(X, ldx, nx2));
    if (!std::isfinite(nx2)) return fail(h, RESPCA_ERR_NONFINITE, "X contains NaN or Inf");
    launch_zero2d<T>(L, ldl, d, n, st);
    launch_zero2d<T>(S, lds, d, n, st);   // S = Theta = 0, or B = 0
    if (!compact) launch_zero2d<T>(Th, d, d, n, st);
    if (nx2 == 0.0) {
        if (labels) launch_zero_i32(labels, n, st);
        CK(hipStreamSynchronize(st));
        info->status = RESPCA_OK;
        return RESPCA_OK;
    }
    const double nX = std::sqrt(nx2);

    if (r.init_embedding && r.emb_refine == 2) {
        // the embedding places the k-means++ seeds; their columns of X start the
        // K-means of X (as without an embedding)
        {
            Engine<float> ez{h, st, r.emb_rows, n, r.c, false};
            CKS(ez.setup());
            CKS(ez.place_seeds(r.init_embedding, r.emb_ld, r.seed));
        }
        CKS(e.setup());
        int steps = 0;
        CKS(e.from_seeds(X, ldx, r.max_lloyd, C, cur, alt, steps));
        info->init_lloyd = steps;
    } else if (r.init_embedding) {
        // groups from K-means of the embedding's columns, then as with init labels
        CKS(ensure(h, h->embl, n * sizeof(int32_t)));
        CKS(ensure(h, h->embc, (size_t)r.emb_rows * r.c * sizeof(float)));
        int steps = 0;
        CKS(kmeans_f32(h, r.emb_rows, n, r.c, r.init_embedding, r.emb_ld, r.seed, r.max_lloyd,
                       (int32_t*)h->embl.p, (float*)h->embc.p, st, &steps));
        CKS(e.setup());
        CK(hipMemcpyAsync(cur, h->embl.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        // Lloyd on the columns of X from the means of X over those groups (empty at zero)
        int ref = 0;
        if (r.emb_refine) {
            launch_zero2d<T>(C, d, d, r.c, st);
            double* gs = nullptr;
            CKS(e.group_sums(gs));
            e.sort(cur);
            e.group_means(false, X, ldx, nullptr, 0, nullptr, 0, T(0), C, gs);
            CKS(e.lloyd(X, ldx, C, cur, alt, r.max_lloyd, ref, nullptr, true));
        }
        info->init_lloyd = steps + ref;
        // then as with given initial labels
        launch_zero2d<T>(C, d, d, r.c, st);
        e.sort(cur);
        e.group_means(false, X, ldx, nullptr, 0, nullptr, 0, T(0), C);
    } else if (r.init_labels) {
        std::vector<int32_t> hl(n);
        CK(hipMemcpyAsync(hl.data(), r.init_labels, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (int64_t j = 0; j < n; ++j)
            if (hl[j] < 0 || hl[j] >= r.c) return fail(h, RESPCA_ERR_INVALID, "init_labels out of range");
        CK(hipMemcpyAsync(cur, r.init_labels, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        launch_zero2d<T>(C, d, d, r.c, st);
        e.sort(cur);
        e.group_means(false, X, ldx, nullptr, 0, nullptr, 0, T(0), C);
    } else if (r.pstep == RESPCA_PSTEP_SPECTRAL) {
        // spectral clustering of X's columns, then as with given initial labels
        int steps = 0;
        CKS(e.spectral_groups(r, X, ldx, true, cur, alt, steps));
        info->init_lloyd = steps;
        launch_zero2d<T>(C, d, d, r.c, st);
        e.sort(cur);
        e.group_means(false, X, ldx, nullptr, 0, nullptr, 0, T(0), C);
    } else {
        int steps = 0;
        CKS(e.kmeans(X, ldx, r.seed, r.max_lloyd, C, cur, alt, steps));
        info->init_lloyd = steps;
    }

    double rho = r.rho0;
    double rho_prev = r.rho0;   // B = 0 stands for S = Theta = 0 at any penalty
    info->status = RESPCA_NOT_CONVERGED;
    for (int t = 1; t <= r.max_iter; ++t) {
        double norms[3];
        int steps = 0;
        CKS(e.iterate_once(r, X, ldx, L, ldl, S, lds, Th, d, C, cur, alt, rho, norms, steps,
                           compact ? rho_prev : 0.0));
        rho_prev = rho;
        info->lloyd_steps += steps;
        info->iters = t;
        info->rho_final = rho;
        info->primal = norms[0] / nX;
        info->dL = norms[1] / nX;
        info->dS = norms[2] / nX;
        if (r.history) {
            r.history[3 * (t - 1) + 0] = info->primal;
            r.history[3 * (t - 1) + 1] = info->dL;
            r.history[3 * (t - 1) + 2] = info->dS;
        }
        const double next = r.kappa * rho;
        rho = next < r.rho_max ? next : r.rho_max;
        const double crit = std::fmax(info->primal, std::fmax(info->dL, info->dS));
        if (crit <= r.tol) {
            info->status = RESPCA_OK;
            break;
        }
    }
    // S of the last iteration from its B, with the threshold that iteration used
    if (compact) launch_soft_inplace<T>(S, lds, d, n, 1.0 / rho_prev, st);
    if (labels) CK(hipMemcpyAsync(labels, cur, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    CK(hipStreamSynchronize(st));
    info->refined = e.refined;
    info->eig_iters = (int32_t)e.spec.iters;
    info->eig_unconverged = (int32_t)e.spec.unconverged;
    return (respca_status)info->status;
}

template <typename T>
respca_status iterate_t(respca_handle h, const Resolved& r, int64_t d, int64_t n, const T* X,
                        int64_t ldx, T* L, int64_t ldl, T* S, int64_t lds, T* Th, int64_t ldt,
                        int32_t* labels, T* C, double* rho, int iters, double* norms_out,
                        respca_info* info, hipStream_t st) {
    Engine<T> e{h, st, d, n, r.c, r.precision == RESPCA_BF16GEMM_F32};
    CKS(e.setup());
    int32_t* cur = (int32_t*)h->lab_a.p;
    int32_t* alt = (int32_t*)h->lab_b.p;
    {
        std::vector<int32_t> hl(n);
        CK(hipMemcpyAsync(hl.data(), labels, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (int64_t j = 0; j < n; ++j)
            if (hl[j] < 0 || hl[j] >= r.c) return fail(h, RESPCA_ERR_INVALID, "labels out of range");
    }
    CK(hipMemcpyAsync(cur, labels, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    double rr = *rho;
    for (int t = 0; t < iters; ++t) {
        double norms[3];
        int steps = 0;
        CKS(e.iterate_once(r, X, ldx, L, ldl, S, lds, Th, ldt, C, cur, alt, rr, norms, steps));
        info->lloyd_steps += steps;
        info->iters = t + 1;
        info->rho_final = rr;
        if (norms_out) std::memcpy(norms_out + 3 * t, norms, sizeof(norms));
        const double next = r.kappa * rr;
        rr = next < r.rho_max ? next : r.rho_max;
    }
    *rho = rr;
    CK(hipMemcpyAsync(labels, cur, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    CK(hipStreamSynchronize(st));
    info->refined = e.refined;
    info->eig_iters = (int32_t)e.spec.iters;
    info->eig_unconverged = (int32_t)e.spec.unconverged;
    info->status = RESPCA_OK;
    return RESPCA_OK;
}

template <typename T>
respca_status kmeans_t(respca_handle h, const Resolved& r, int64_t d, int64_t n, const T* Y,
                       int64_t ldy, int32_t* labels, T* C, respca_info* info, hipStream_t st) {
    Engine<T> e{h, st, d, n, r.c, r.precision == RESPCA_BF16GEMM_F32};
    CKS(e.setup());
    int32_t* cur = (int32_t*)h->lab_a.p;
    int32_t* alt = (int32_t*)h->lab_b.p;
    int steps = 0;
    CKS(e.kmeans(Y, ldy, r.seed, r.max_lloyd, C, cur, alt, steps));
    info->init_lloyd = steps;
    CK(hipMemcpyAsync(labels, cur, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    CK(hipStreamSynchronize(st));
    info->refined = e.refined;
    info->status = RESPCA_OK;
    return RESPCA_OK;
}

}  // namespace

respca_status respca::kmeans_f32(respca_handle h, int64_t d, int64_t n, int c, const float* Y,
                                 int64_t ldy, uint64_t seed, int max_lloyd, int32_t* labels, float* C,
                                 hipStream_t st, int* steps) {
    Engine<float> e{h, st, d, n, c, false};
    CKS(e.setup());
    int32_t* cur = (int32_t*)h->lab_a.p;
    int32_t* alt = (int32_t*)h->lab_b.p;
    int s = 0;
    CKS(e.kmeans(Y, ldy, seed, max_lloyd, C, cur, alt, s));
    if (steps) *steps = s;
    CK(hipMemcpyAsync(labels, cur, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    return RESPCA_OK;
}

namespace {

respca_status bind_device(respca_handle h) {
    CK(hipSetDevice(h->device));
    return RESPCA_OK;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

respca_status respca_create(respca_handle* out, int32_t device) {
    if (!out) return RESPCA_ERR_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return RESPCA_ERR_HIP;
    auto* h = new (std::nothrow) respca_handle_s();
    if (!h) return RESPCA_ERR_NOMEM;
    h->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return RESPCA_ERR_HIP;
    }
    // The scratch address of this device; on failure respca_iterate_noalloc
    // retries and reports the error, every other entry point works without it.
    if (lookup_scratch(h, device) != RESPCA_OK) (void)hipGetLastError();
    h->err.clear();
    *out = h;
    return RESPCA_OK;
}

void respca_destroy(respca_handle h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    for (auto& p : h->prof_pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : h->prof_pool) (void)hipEventDestroy(e);
    if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
    if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
    if (h->bev) (void)hipEventDestroy(h->bev);
    if (h->bstream) (void)hipStreamDestroy(h->bstream);
    if (h->bws.p) (void)hipFree(h->bws.p);
    if (h->bstage) (void)hipHostFree(h->bstage);
    respca::DevBuf* wbufs[] = {&h->wsk, &h->wfeat, &h->wacts, &h->wscratch, &h->wred, &h->wcent,
                               &h->embl, &h->embc, &h->wdesc, &h->whash, &h->probe,
                               &h->sp_w, &h->sp_q, &h->sp_s, &h->sp_y, &h->sp_z, &h->sp_yp,
                               &h->sp_t, &h->sp_part, &h->sp_small, &h->sp_emb, &h->sp_cent,
                               &h->sp_mean};
    for (respca::DevBuf* b : wbufs)
        if (b->p) (void)hipFree(b->p);
    DevBuf* bufs[] = {&h->theta, &h->cbuf, &h->perm, &h->counts, &h->segb, &h->segl, &h->segf,
                      &h->nseg, &h->sortbc, &h->pmeans, &h->dots, &h->cnorm, &h->lab_a, &h->lab_b, &h->d2,
                      &h->zcopy, &h->zsc, &h->ynorm, &h->gsum, &h->cnt2, &h->cbc, &h->cperm,
                      &h->csegb, &h->csegl, &h->csegf, &h->cnseg, &h->cpart,
                      &h->chosen, &h->seeds, &h->u, &h->normp, &h->chgp, &h->status};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (h->hstage) (void)hipHostFree(h->hstage);
    if (h->hstatus) (void)hipHostFree(h->hstatus);
    if (h->sp_status) (void)hipHostFree(h->sp_status);
    delete h;
}

void respca_params_default(respca_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->lambda = NAN;
    p->rank = 0;
    p->tol = 1e-3;
    p->max_iter = 500;
    p->rho0 = 1e-4;
    p->kappa = 1.5;
    p->rho_max = 1e10;
    p->max_lloyd = 100;
    p->seed = 0;
    p->precision = RESPCA_F32;
    p->sparse_norm = RESPCA_SPARSE_L1;
    p->init_labels = nullptr;
    p->history = nullptr;
    p->init_embedding = nullptr;
    p->init_embedding_ld = 0;
    p->init_embedding_rows = 0;
    p->pstep = RESPCA_PSTEP_KMEANS;
    p->spectral_sigma = 0.0;
    p->init_embedding_refine = 1;
}

const char* respca_status_string(respca_status s) {
    switch (s) {
        case RESPCA_OK: return "RESPCA_OK";
        case RESPCA_NOT_CONVERGED: return "RESPCA_NOT_CONVERGED";
        case RESPCA_ERR_INVALID: return "RESPCA_ERR_INVALID";
        case RESPCA_ERR_NONFINITE: return "RESPCA_ERR_NONFINITE";
        case RESPCA_ERR_NOMEM: return "RESPCA_ERR_NOMEM";
        case RESPCA_ERR_HIP: return "RESPCA_ERR_HIP";
        case RESPCA_ERR_UNSUPPORTED: return "RESPCA_ERR_UNSUPPORTED";
    }
    return "unknown status";
}

const char* respca_last_error(respca_handle h) { return h ? h->err.c_str() : "NULL handle"; }

const char* respca_version(void) { return kVersion; }

respca_status respca_profile_enable(respca_handle h, int32_t enable) {
    if (!h) return RESPCA_ERR_INVALID;
    if (hipSetDevice(h->device) != hipSuccess) return RESPCA_ERR_HIP;
    if (!h->prof_pending.empty()) {
        (void)hipDeviceSynchronize();
        prof_resolve(h);
    }
    h->prof_mask = (uint32_t)enable;
    h->prof_on = enable != 0;
    for (int k = 0; k < RESPCA_KERNEL_COUNT; ++k) {
        h->prof_launches[k] = 0;
        h->prof_ms[k] = 0.0;
        h->prof_bytes[k] = 0.0;
        h->prof_flops[k] = 0.0;
    }
    return RESPCA_OK;
}

respca_status respca_profile_query(respca_handle h, int32_t kernel, int64_t* launches,
                                   double* total_ms, double* bytes, double* flops) {
    if (!h || kernel < 0 || kernel >= RESPCA_KERNEL_COUNT) return RESPCA_ERR_INVALID;
    if (!h->prof_pending.empty()) {
        if (hipSetDevice(h->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return RESPCA_ERR_HIP;
        prof_resolve(h);
    }
    if (launches) *launches = h->prof_launches[kernel];
    if (total_ms) *total_ms = h->prof_ms[kernel];
    if (bytes) *bytes = h->prof_bytes[kernel];
    if (flops) *flops = h->prof_flops[kernel];
    return RESPCA_OK;
}

respca_status respca_solve(respca_handle h, const respca_params* params, int64_t d, int64_t n,
                           const void* X, int64_t ldx, void* L, int64_t ldl, void* S, int64_t lds,
                           int32_t* labels, respca_info* info, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    respca_info local{};
    respca_info* out = info ? info : &local;
    std::memset(out, 0, sizeof(*out));
    Resolved r;
    respca_status s = resolve(h, params, d, n, r);
    if (s == RESPCA_OK) {
        const size_t w = r.precision == RESPCA_F64 ? 8 : 4;
        if (!X || !L || !S) s = fail(h, RESPCA_ERR_INVALID, "X, L and S must be non-NULL");
        else if (ldx < d || ldl < d || lds < d) s = fail(h, RESPCA_ERR_INVALID, "leading dimension < d");
        else {
            Span sx = span_of(X, ldx, d, n, w), sl = span_of(L, ldl, d, n, w), ss = span_of(S, lds, d, n, w);
            if (overlap(sx, sl) || overlap(sx, ss) || overlap(sl, ss))
                s = fail(h, RESPCA_ERR_INVALID, "X, L and S must not overlap");
        }
    }
    if (s == RESPCA_OK) s = bind_device(h);
    if (s == RESPCA_OK) {
        hipStream_t st = (hipStream_t)stream;
        if (r.precision == RESPCA_F64)
            s = solve_t<double>(h, r, d, n, (const double*)X, ldx, (double*)L, ldl, (double*)S, lds,
                                labels, out, st);
        else
            s = solve_t<float>(h, r, d, n, (const float*)X, ldx, (float*)L, ldl, (float*)S, lds,
                               labels, out, st);
    }
    out->status = s;
    return s;
}

}  // extern "C"

namespace {

// Argument checks of respca_iterate and respca_iterate_noalloc.
respca_status check_iterate(respca_handle h, const respca_params* params, int64_t d, int64_t n,
                            const void* X, int64_t ldx, void* L, int64_t ldl, void* S, int64_t lds,
                            void* Theta, int64_t ldt, int32_t* labels, void* C, double* rho,
                            int32_t iters, Resolved& r) {
    respca_status s = resolve(h, params, d, n, r);
    if (s == RESPCA_OK) {
        const size_t w = r.precision == RESPCA_F64 ? 8 : 4;
        if (!X || !L || !S || !Theta || !labels || !C || !rho)
            s = fail(h, RESPCA_ERR_INVALID, "NULL argument");
        else if (ldx < d || ldl < d || lds < d || ldt < d)
            s = fail(h, RESPCA_ERR_INVALID, "leading dimension < d");
        else if (iters < 0)
            s = fail(h, RESPCA_ERR_INVALID, "iters must be >= 0");
        else if (!(*rho > 0.0) || !std::isfinite(*rho))
            s = fail(h, RESPCA_ERR_INVALID, "rho must be > 0");
        else {
            Span sx = span_of(X, ldx, d, n, w), sl = span_of(L, ldl, d, n, w),
                 ss = span_of(S, lds, d, n, w), sth = span_of(Theta, ldt, d, n, w);
            if (overlap(sx, sl) || overlap(sx, ss) || overlap(sl, ss) || overlap(sth, sx) ||
                overlap(sth, sl) || overlap(sth, ss))
                s = fail(h, RESPCA_ERR_INVALID, "X, L, S and Theta must not overlap");
        }
    }
    return s;
}

respca_status run_iterate(respca_handle h, const Resolved& r, int64_t d, int64_t n, const void* X,
                          int64_t ldx, void* L, int64_t ldl, void* S, int64_t lds, void* Theta,
                          int64_t ldt, int32_t* labels, void* C, double* rho, int32_t iters,
                          double* norms, respca_info* out, hipStream_t st) {
    if (r.precision == RESPCA_F64)
        return iterate_t<double>(h, r, d, n, (const double*)X, ldx, (double*)L, ldl, (double*)S,
                                 lds, (double*)Theta, ldt, labels, (double*)C, rho, iters, norms,
                                 out, st);
    return iterate_t<float>(h, r, d, n, (const float*)X, ldx, (float*)L, ldl, (float*)S, lds,
                            (float*)Theta, ldt, labels, (float*)C, rho, iters, norms, out, st);
}

// Workspace buffers of the single-solve engine.  While a no-alloc call runs,
// the handle's own (allocated) buffers are set aside and these point into the
// scratch area; they are put back when the call returns, so the other entry
// points never see (or free) scratch memory.
struct ArenaScope {
    respca_handle h;
    std::vector<DevBuf*> bufs;
    std::vector<DevBuf> saved;
    explicit ArenaScope(respca_handle h_) : h(h_) {
        bufs = {&h->theta, &h->cbuf, &h->perm, &h->counts, &h->segb, &h->segl, &h->segf,
                &h->nseg, &h->sortbc, &h->pmeans, &h->dots, &h->cnorm, &h->lab_a, &h->lab_b,
                &h->d2, &h->chosen, &h->seeds, &h->u, &h->normp, &h->chgp, &h->status,
                &h->l21f, &h->zcopy, &h->zsc, &h->ynorm, &h->gsum, &h->cnt2, &h->cbc,
                &h->cperm, &h->csegb, &h->csegl, &h->csegf, &h->cnseg, &h->cpart};
        for (DevBuf* b : bufs) saved.push_back(*b);
    }
    // Start carving from base (nullptr: a measuring pass that launches nothing).
    void begin(char* base, size_t cap) {
        for (DevBuf* b : bufs) *b = DevBuf{};
        h->arena_on = true;
        h->arena_base = base;
        h->arena_cap = cap;
        h->arena_off = 0;
    }
    ~ArenaScope() {
        for (size_t i = 0; i < bufs.size(); ++i) *bufs[i] = saved[i];
        h->arena_on = false;
        h->arena_base = nullptr;
        h->arena_cap = 0;
        h->arena_off = 0;
    }
};

template <typename T>
respca_status reserve_iterate_t(respca_handle h, const Resolved& r, int64_t d, int64_t n) {
    Engine<T> e{h, nullptr, d, n, r.c, r.precision == RESPCA_BF16GEMM_F32};
    return e.reserve_iterate(r);
}

}  // namespace

extern "C" {

respca_status respca_iterate(respca_handle h, const respca_params* params, int64_t d, int64_t n,
                             const void* X, int64_t ldx, void* L, int64_t ldl, void* S, int64_t lds,
                             void* Theta, int64_t ldt, int32_t* labels, void* C, double* rho,
                             int32_t iters, double* norms, respca_info* info, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    respca_info local{};
    respca_info* out = info ? info : &local;
    std::memset(out, 0, sizeof(*out));
    Resolved r;
    respca_status s = check_iterate(h, params, d, n, X, ldx, L, ldl, S, lds, Theta, ldt, labels, C,
                                    rho, iters, r);
    if (s == RESPCA_OK) s = bind_device(h);
    if (s == RESPCA_OK)
        s = run_iterate(h, r, d, n, X, ldx, L, ldl, S, lds, Theta, ldt, labels, C, rho, iters,
                        norms, out, (hipStream_t)stream);
    out->status = s;
    return s;
}

respca_status respca_iterate_noalloc(respca_handle h, const respca_params* params, int64_t d,
                                     int64_t n, const void* X, int64_t ldx, void* L, int64_t ldl,
                                     void* S, int64_t lds, void* Theta, int64_t ldt,
                                     int32_t* labels, void* C, double* rho, int32_t iters,
                                     double* norms, respca_info* info, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    respca_info local{};
    respca_info* out = info ? info : &local;
    std::memset(out, 0, sizeof(*out));
    Resolved r;
    respca_status s = check_iterate(h, params, d, n, X, ldx, L, ldl, S, lds, Theta, ldt, labels, C,
                                    rho, iters, r);
    if (s == RESPCA_OK) s = bind_device(h);
    if (s == RESPCA_OK && h->device >= kMaxScratchDevices)
        s = fail(h, RESPCA_ERR_UNSUPPORTED, "no scratch area for device ordinals above 63");
    if (s == RESPCA_OK && r.pstep != RESPCA_PSTEP_KMEANS)
        s = fail(h, RESPCA_ERR_UNSUPPORTED, "the no-alloc entry point runs the K-means p-step only");
    if (s == RESPCA_OK) s = lookup_scratch(h, h->device);
    if (s == RESPCA_OK) {
        char* base = nullptr;
        {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            base = g_scratch_ptr[h->device];
        }
        ArenaScope arena(h);
        // measure first, so that a problem too large fails before any work is enqueued
        arena.begin(nullptr, ~(size_t)0 >> 1);
        s = r.precision == RESPCA_F64 ? reserve_iterate_t<double>(h, r, d, n)
                                      : reserve_iterate_t<float>(h, r, d, n);
        const size_t need = h->arena_off;
        if (s == RESPCA_OK && need > (size_t)RESPCA_NOALLOC_SCRATCH_BYTES)
            s = fail(h, RESPCA_ERR_UNSUPPORTED,
                     "problem needs " + std::to_string(need) + " bytes of scratch, the maximum is " +
                         std::to_string((size_t)RESPCA_NOALLOC_SCRATCH_BYTES));
        if (s == RESPCA_OK) {
            arena.begin(base, RESPCA_NOALLOC_SCRATCH_BYTES);
            s = r.precision == RESPCA_F64 ? reserve_iterate_t<double>(h, r, d, n)
                                          : reserve_iterate_t<float>(h, r, d, n);
        }
        if (s == RESPCA_OK)
            s = run_iterate(h, r, d, n, X, ldx, L, ldl, S, lds, Theta, ldt, labels, C, rho, iters,
                            norms, out, (hipStream_t)stream);
    }
    out->status = s;
    return s;
}

respca_status respca_spectral_embedding(respca_handle h, int32_t precision, int64_t d, int64_t n,
                                        const void* Y, int64_t ldy, int32_t c, double sigma,
                                        uint64_t seed, double* emb, double* eigenvalues,
                                        respca_info* info, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    respca_info local{};
    respca_info* out = info ? info : &local;
    std::memset(out, 0, sizeof(*out));
    respca_status s = RESPCA_OK;
    if (!Y || !emb) s = fail(h, RESPCA_ERR_INVALID, "NULL argument");
    else if (d < 1 || n < 2 || d >= (int64_t)INT32_MAX || ldy < d)
        s = fail(h, RESPCA_ERR_INVALID, "need d >= 1, n >= 2, ldy >= d");
    else if (c < 1 || c >= n) s = fail(h, RESPCA_ERR_INVALID, "c must be in [1, n)");
    else if (sigma == 0.0 || !std::isfinite(sigma))
        s = fail(h, RESPCA_ERR_INVALID, "sigma must be finite and nonzero");
    else if (precision != RESPCA_F64 && precision != RESPCA_F32 && precision != RESPCA_BF16GEMM_F32)
        s = fail(h, RESPCA_ERR_INVALID, "unknown precision");
    else if (c > kSpectralMaxGroups || n > kSpectralMaxN)
        s = fail(h, RESPCA_ERR_UNSUPPORTED, "spectral embedding: c <= 40 and n <= 32768");
    if (s == RESPCA_OK) s = bind_device(h);
    if (s == RESPCA_OK) {
        hipStream_t st = (hipStream_t)stream;
        SpectralStats stats;
        s = precision == RESPCA_F64
                ? spectral_embed<double>(h, (const double*)Y, ldy, d, n, c, sigma, seed, emb, &stats, st)
                : spectral_embed<float>(h, (const float*)Y, ldy, d, n, c, sigma, seed, emb, &stats, st);
        if (s == RESPCA_OK && eigenvalues) s = spectral_eigenvalues(h, n, c, eigenvalues, st);
        if (s == RESPCA_OK) {
            if (hipStreamSynchronize(st) != hipSuccess) s = fail(h, RESPCA_ERR_HIP, "stream sync failed");
            prof_resolve(h);
        }
        out->eig_iters = (int32_t)stats.iters;
        out->eig_unconverged = (int32_t)stats.unconverged;
    }
    out->status = s;
    return s;
}

respca_status respca_kmeans(respca_handle h, const respca_params* params, int64_t d, int64_t n,
                            const void* Y, int64_t ldy, int32_t* labels, void* C,
                            respca_info* info, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    respca_info local{};
    respca_info* out = info ? info : &local;
    std::memset(out, 0, sizeof(*out));
    Resolved r;
    respca_status s = resolve(h, params, d, n, r);
    if (s == RESPCA_OK) {
        if (!Y || !labels || !C) s = fail(h, RESPCA_ERR_INVALID, "NULL argument");
        else if (ldy < d) s = fail(h, RESPCA_ERR_INVALID, "leading dimension < d");
    }
    if (s == RESPCA_OK) s = bind_device(h);
    if (s == RESPCA_OK) {
        hipStream_t st = (hipStream_t)stream;
        if (r.precision == RESPCA_F64)
            s = kmeans_t<double>(h, r, d, n, (const double*)Y, ldy, labels, (double*)C, out, st);
        else
            s = kmeans_t<float>(h, r, d, n, (const float*)Y, ldy, labels, (float*)C, out, st);
    }
    out->status = s;
    return s;
}

}  // extern "C"
