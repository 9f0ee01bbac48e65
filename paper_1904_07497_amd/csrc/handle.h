// Handle state and host-side helpers shared by the library's host files
// (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/respca.h"

namespace respca {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct ProfPending {
    int kernel;
    hipEvent_t a, b;
    double bytes, flops;
};

// Tile shapes of the batched solver (set by the tuner, or these defaults).
struct BatchTune {
    int jc = 8;             // columns per sweep / pack work item
    int slice_rows = 1024;  // rows per distance slice (multiple of 32)
    int blocks_per_cu = 2;  // persistent workgroups per compute unit
};

}  // namespace respca

struct respca_handle_s {
    int device = 0;
    std::string err;
    // kernel timing
    bool prof_on = false;     // some unit is timed
    uint32_t prof_mask = 0;   // bit k: launches of kernel id k are timed
    int64_t prof_launches[RESPCA_KERNEL_COUNT] = {};
    double prof_ms[RESPCA_KERNEL_COUNT] = {};
    double prof_bytes[RESPCA_KERNEL_COUNT] = {};
    double prof_flops[RESPCA_KERNEL_COUNT] = {};
    std::vector<respca::ProfPending> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    respca::DevBuf theta, cbuf, perm, counts, segb, segl, segf, nseg, sortbc, pmeans, dots, cnorm,
        lab_a, lab_b, d2, chosen, seeds, u, normp, chgp, status;
    respca::DevBuf l21f;                // per-column l2,1 S-step factors (n doubles)
    respca::DevBuf zcopy, zsc, ynorm;   // fp16 copy, column scales and norms for bounded seeding
    // incremental Lloyd means: group sums, next counts, the moved-column sort and its partials
    respca::DevBuf gsum, cnt2, cbc, cperm, csegb, csegl, csegf, cnseg, cpart;
    double* hstage = nullptr;  // pinned host staging (uniforms, small copies)
    // Pinned host copy of the status words (words 0..7) and the sequence number of
    // the last copy (word 8), written by the device after the words; the host
    // polls word 8 instead of synchronizing the stream.
    double* hstatus = nullptr;
    double* hstatus_dev = nullptr;  // the same memory as the device sees it
    uint64_t status_seq = 0;        // last sequence number asked for
    size_t hstage_bytes = 0;
    // batched solver
    respca::BatchTune tune;
    respca::DevBuf bws;             // batched workspace (descriptors, tables, instance arrays)
    char* bstage = nullptr;         // pinned staging of descriptors/tables/uniforms + readback
    size_t bstage_bytes = 0;
    hipStream_t bstream = nullptr;  // internal stream (graph capture needs a non-null stream)
    hipEvent_t bev = nullptr;
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bexec = nullptr;
    uint64_t bsig = 0;              // signature of the captured call
    double bphase_ms[16] = {};      // phase times of the last batched launch
    int64_t bsteps = 0;
    // warm start
    respca::DevBuf wsk, wfeat, wacts, wscratch, wred, wcent, embl, embc, wdesc, whash;
    respca::DevBuf probe;           // arrays of the bandwidth probe
    // spectral p-step: affinity (n x n), norms, scales, eigen blocks, partials,
    // small matrices, the row embedding and its centroids
    respca::DevBuf sp_w, sp_q, sp_s, sp_y, sp_z, sp_yp, sp_t, sp_part, sp_small, sp_emb, sp_cent,
        sp_mean;
    double* sp_status = nullptr;      // pinned host words the eigen loop reads back
    double* sp_status_dev = nullptr;
    // Carving mode of ensure(): while arena_on, buffers are cut from [arena_base,
    // arena_base + arena_cap) instead of allocated (arena_base may be 0 for a
    // measuring pass that launches nothing); arena_off is the bytes used so far.
    bool arena_on = false;
    char* arena_base = nullptr;
    size_t arena_cap = 0, arena_off = 0;
};

#define CK(expr)                                                                            \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            h->err = std::string(#expr) + ": " + hipGetErrorString(e_);                     \
            return e_ == hipErrorOutOfMemory ? RESPCA_ERR_NOMEM : RESPCA_ERR_HIP;           \
        }                                                                                   \
    } while (0)

#define CKS(expr)                                    \
    do {                                             \
        respca_status s_ = (expr);                   \
        if (s_ < 0) return s_;                       \
    } while (0)

namespace respca {

inline respca_status ensure(respca_handle h, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return RESPCA_OK;
    if (h->arena_on) {   // carve (256-byte aligned); never allocates
        const size_t off = (h->arena_off + 255) & ~(size_t)255;
        if (bytes > h->arena_cap || off > h->arena_cap - bytes) {
            h->arena_off = off + bytes;
            h->err = "scratch area too small for this problem";
            return RESPCA_ERR_UNSUPPORTED;
        }
        b.p = h->arena_base + off;
        b.bytes = bytes;
        h->arena_off = off + bytes;
        return RESPCA_OK;
    }
    if (b.p) CK(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    CK(hipMalloc(&b.p, bytes));
    b.bytes = bytes;
    return RESPCA_OK;
}

inline respca_status ensure_host(respca_handle h, size_t bytes) {
    if (h->hstage_bytes >= bytes) return RESPCA_OK;
    if (h->hstage) CK(hipHostFree(h->hstage));
    h->hstage = nullptr;
    h->hstage_bytes = 0;
    CK(hipHostMalloc((void**)&h->hstage, bytes, hipHostMallocDefault));
    h->hstage_bytes = bytes;
    return RESPCA_OK;
}

// Event bracket around one launch (no-op unless timing is enabled).
struct ProfScope {
    respca_handle h;
    hipStream_t st;
    int kernel;
    double bytes, flops;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(respca_handle h_, hipStream_t st_, int k, double by, double fl = 0.0)
        : h(h_), st(st_), kernel(k), bytes(by), flops(fl) {
        // not timed while carving from the fixed scratch area (events are created lazily)
        if (!((h->prof_mask >> kernel) & 1u) || h->arena_on) return;
        a = take();
        b = take();
        if (a && b) (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a || !b) return;
        (void)hipEventRecord(b, st);
        h->prof_pending.push_back({kernel, a, b, bytes, flops});
    }
    hipEvent_t take() {
        if (!h->prof_pool.empty()) {
            hipEvent_t e = h->prof_pool.back();
            h->prof_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

inline respca_status ensure_spectral_status(respca_handle h) {
    if (h->sp_status) return RESPCA_OK;
    CK(hipHostMalloc((void**)&h->sp_status, 8 * sizeof(double), hipHostMallocMapped));
    CK(hipHostGetDevicePointer((void**)&h->sp_status_dev, h->sp_status, 0));
    return RESPCA_OK;
}

inline respca_status fail(respca_handle h, respca_status s, const std::string& msg) {
    if (h) h->err = msg;
    return s;
}

// splitmix64 (Steele, Lea & Flood 2014) and the uniform in [0, 1) from its top 53 bits.
inline uint64_t splitmix64_next(uint64_t& state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

inline double uniform01(uint64_t& state) {
    return (double)(splitmix64_next(state) >> 11) * 0x1.0p-53;
}

// Parameters after defaults are applied.
struct Resolved {
    double lambda, tol, rho0, kappa, rho_max;
    int c, max_iter, max_lloyd, precision, sparse_norm;
    int pstep;
    double sigma;   // spectral p-step kernel width
    uint64_t seed;
    const int32_t* init_labels;
    double* history;
    const float* init_embedding;
    int64_t emb_ld;
    int emb_rows;
    int emb_refine;   // Lloyd on X after the embedding's K-means (1), not (0), or seeding only (2)
};

respca_status resolve(respca_handle h, const respca_params* p, int64_t d, int64_t n, Resolved& r);

// K-means (k-means++ from splitmix64(seed), then Lloyd) of the columns of a
// float d x n matrix; labels (device) and C (device d x c) out; enqueued on st.
respca_status kmeans_f32(respca_handle h, int64_t d, int64_t n, int c, const float* Y, int64_t ldy,
                         uint64_t seed, int max_lloyd, int32_t* labels, float* C, hipStream_t st,
                         int* steps);

}  // namespace respca
