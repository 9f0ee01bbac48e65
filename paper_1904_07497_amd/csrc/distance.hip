// K-means assignment pass (the p-step of Sec. 4.2): for every column Y_j,
// label_j = argmin_k ||C_k||^2 - 2 C_k . Y_j  (||Y_j||^2 is common to all k),
// ties to the lowest k.
//
// FP32 runs: the C^T Y contraction runs on the matrix cores
// (v_mfma_f32_16x16x4f32).  A workgroup owns 128 columns x 128 groups and one
// slice of rows; both operands are staged through LDS 32 rows at a time with
// 16-byte coalesced loads (a column's 32 rows are 128 contiguous bytes), and
// each wave keeps 2 x 8 accumulator tiles of 16 x 16.  Per-slice partial dot
// products go to a [slice][column][group] buffer; a second kernel sums the
// slices in fixed order in double, forms the distances and takes the argmin
// with 16 lanes per column.  FP64 runs use the VALU contraction in kernels.hip.
//
// bf16 mode: the same tiles, but each FP32 operand x is split into
// x_hi = bf16(x) and x_lo = bf16(x - x_hi), and C.Y is accumulated in FP32 as
// hi.hi + hi.lo + lo.hi on v_mfma_f32_16x16x32_bf16 (one instruction covers a
// whole 32-row stage).  The dropped lo.lo term and the rounding of x_lo are
// each below 2^-16 |c||y| per product, so with the FP32 accumulation error a
// distance carries at most E = (3 * 2^-15 + 2 K 2^-24) ||C_k|| ||Y_j|| error
// (K = rows summed in FP32).  The kernel also accumulates ||Y_j||^2; the argmin
// kernel flags every column whose best and runner-up distances are not
// separated by the bounds, and those columns are re-decided exactly (FP64
// differences of the FP32 values) by a refinement kernel.  With 17 to 32
// groups this bounded mode runs the FP32 MFMA tile instead (few MFMAs, no split
// work; E = 2 (K + 2) 2^-24 ||C_k|| ||Y_j|| from the FP32 products and sums) with
// the same argmin and refinement, so its labels are exact as well.  With at most
// 16 groups it accumulates the products in FP64 on the vector units (the FP64
// tile below): the distances are then FP64 ones and nothing is refined.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "kernels.h"
#include "dist_tile.h"

namespace respca {

namespace {

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// bf16, VEC: the direct tile, 8 waves x 32 columns and NKB group blocks per
// workgroup (one workgroup per CU: the 256 columns share each centroid stage).
constexpr int kDirectWaves = 8;
constexpr int kJD = 32 * kDirectWaves;   // columns per direct workgroup

// Up to three group blocks the registers fit two workgroups per CU (four waves
// per SIMD); more blocks take one.
constexpr int direct_wgs_per_cu(int nkb) { return nkb <= 3 ? 2 : 1; }

template <int NKB>
__global__ __launch_bounds__(64 * kDirectWaves) __attribute__((amdgpu_waves_per_eu(2 * direct_wgs_per_cu(NKB), 2 * direct_wgs_per_cu(NKB)))) void k_dist_mfma_direct(
    int64_t d, int c, int kpad, const float* __restrict__ Y, int64_t ldy, int64_t n, int slice_rows,
    float* __restrict__ part, float* __restrict__ ynorm_part, int* __restrict__ counters,
    const uint4* __restrict__ Csp, int64_t ldq) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x < 4)
        counters[threadIdx.x] = 0;   // refinement list length, its changed count: fresh for this pass
    // one workgroup per CU: two stages of column values in flight per wave (eight
    // group blocks leave no registers for the second)
    dist_tile_ydirect<NKB, kDirectWaves, direct_wgs_per_cu(NKB) == 1 && NKB < 8 ? 2 : 1>(
        d, kpad, Y, ldy, n, slice_rows, part, ynorm_part, (int64_t)blockIdx.x * kJD, blockIdx.y,
        blockIdx.z * kKC, blockIdx.z == 0, Csp, ldq);
}

// Bounded mode at small c: the FP32 MFMA tile with the columns' norms, decided by
// the same bounded argmin and exact refinement as the split-bf16 tiles.
template <bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_dist_mfma_f32b(
    const float* __restrict__ C, int64_t d, int c, int kpad, const float* __restrict__ Y, int64_t ldy,
    int64_t n, int slice_rows, float* __restrict__ part, float* __restrict__ ynorm_part,
    int* __restrict__ counters) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x < 4)
        counters[threadIdx.x] = 0;   // refinement list length, its changed count: fresh for this pass
    dist_tile<VEC, false, true, false, true>(C, d, c, kpad, Y, ldy, n, slice_rows, part, ynorm_part,
                                             (int64_t)blockIdx.x * kJT, blockIdx.y, blockIdx.z * kKC,
                                             blockIdx.z == 0);
}

template <bool VEC, bool BF16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_dist_mfma(const float* __restrict__ C, int64_t d, int c,
                                                   int kpad, const float* __restrict__ Y, int64_t ldy,
                                                   int64_t n, int slice_rows,
                                                   float* __restrict__ part,
                                                   float* __restrict__ ynorm_part,
                                                   int* __restrict__ counters,
                                                   const uint4* __restrict__ Csp, int64_t ldq) {
    if (BF16 && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x < 4)
        counters[threadIdx.x] = 0;   // refinement list length, its changed count: fresh for this pass
    dist_tile<VEC, BF16, true, BF16>(C, d, c, kpad, Y, ldy, n, slice_rows, part, ynorm_part,
                                     (int64_t)blockIdx.x * kJT, blockIdx.y, blockIdx.z * kKC,
                                     blockIdx.z == 0, Csp, ldq);
}

// bf16 mode, once per pass: every centroid split into its bf16 parts in the
// layout the distance tile stages from (rows 4g..4g+3 of group k as {hi[4],
// lo[4]} at Csp[k * ldq + g], zero past row d and for the padding groups
// c..kpad-1), and cnorm[k] = ||C_k||^2 in double.  One workgroup per group.
__global__ __launch_bounds__(1024) void k_split_centroids(const float* __restrict__ C, int64_t d,
                                                          int c, int64_t ldq, bool vec,
                                                          uint4* __restrict__ Csp,
                                                          double* __restrict__ cnorm) {
    const int k = blockIdx.x;
    const float* ck = C + (int64_t)k * d;
    double a = 0.0;
    for (int64_t g = threadIdx.x; g < ldq; g += 1024) {
        float x[4] = {0.f, 0.f, 0.f, 0.f};
        if (k < c && 4 * g < d) {
            if (vec) {   // d % 4 == 0 and C 16-byte aligned: one load per row group
                const float4 t = *reinterpret_cast<const float4*>(ck + 4 * g);
                x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * g + e < d) x[e] = ck[4 * g + e];
            }
        }
        bf16x4 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            h[e] = (__bf16)x[e];
            l[e] = (__bf16)(x[e] - (float)h[e]);
            a += (double)x[e] * (double)x[e];
        }
        uint4 v;
        const uint2 hb = *reinterpret_cast<const uint2*>(&h), lb = *reinterpret_cast<const uint2*>(&l);
        v.x = hb.x; v.y = hb.y; v.z = lb.x; v.w = lb.y;
        Csp[(int64_t)k * ldq + g] = v;
    }
    a = wave_sum_d(a);
    __shared__ double sh[16];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0 && k < c) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += sh[w];
        cnorm[k] = t;
    }
}

// 16 lanes per column: lane q takes groups q, q+16, ...; slices summed in order
// in double; (distance, group) lexicographic minimum across the 16 lanes.
__global__ __launch_bounds__(256) void k_dist_argmin(const float* __restrict__ part, int nslices,
                                                     int64_t n, int c, int kpad,
                                                     const double* __restrict__ cnorm,
                                                     const int32_t* __restrict__ old_labels,
                                                     int32_t* __restrict__ new_labels,
                                                     double* __restrict__ changed_partial) {
    __shared__ double sh[4];
    const int q = threadIdx.x & 15;
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    double bestd = INFINITY;
    int bestk = INT_MAX;
    if (j < n) {
        for (int k = q; k < c; k += 16) {
            double dot = 0.0;
            for (int s = 0; s < nslices; ++s) dot += (double)part[((int64_t)s * n + j) * kpad + k];
            const double dist = cnorm[k] - 2.0 * dot;
            if (dist < bestd) { bestd = dist; bestk = k; }
        }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        const double od = __shfl_xor(bestd, o, 16);
        const int ok = __shfl_xor(bestk, o, 16);
        if (od < bestd || (od == bestd && ok < bestk)) { bestd = od; bestk = ok; }
    }
    double changed = 0.0;
    if (j < n && q == 0) {
        const int lab = bestk == INT_MAX ? 0 : bestk;
        new_labels[j] = lab;
        changed = old_labels[j] != lab ? 1.0 : 0.0;
    }
    changed = wave_sum_d(changed);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = changed;
    __syncthreads();
    if (threadIdx.x == 0) changed_partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// FP32 mode, c <= 16 T: the same minimum with each lane's T group sums held in
// registers (slices summed in the same order).
template <int T>
__global__ __launch_bounds__(256) void k_dist_argmin_r(const float* __restrict__ part, int nslices,
                                                       int64_t n, int c, int kpad,
                                                       const double* __restrict__ cnorm,
                                                       const int32_t* __restrict__ old_labels,
                                                       int32_t* __restrict__ new_labels,
                                                       double* __restrict__ changed_partial) {
    __shared__ double sh[4];
    const int q = threadIdx.x & 15;
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool live = j < n;
    double dot[T], ynorm;
    sum_slices<T, false>(part, nullptr, live ? nslices : 0, n, j, c, kpad, q, dot, ynorm);
    double bestd = INFINITY;
    int bestk = INT_MAX;
    double cn[T];   // loaded unconditionally (clamped), used only below c
#pragma unroll
    for (int t = 0; t < T; ++t) cn[t] = cnorm[q + 16 * t < c ? q + 16 * t : c - 1];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int k = q + 16 * t;
        if (live && k < c) {
            const double dist = cn[t] - 2.0 * dot[t];
            if (dist < bestd) { bestd = dist; bestk = k; }
        }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        const double od = __shfl_xor(bestd, o, 16);
        const int ok = __shfl_xor(bestk, o, 16);
        if (od < bestd || (od == bestd && ok < bestk)) { bestd = od; bestk = ok; }
    }
    double changed = 0.0;
    if (live && q == 0) {
        const int lab = bestk == INT_MAX ? 0 : bestk;
        new_labels[j] = lab;
        changed = old_labels[j] != lab ? 1.0 : 0.0;
    }
    changed = wave_sum_d(changed);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = changed;
    __syncthreads();
    if (threadIdx.x == 0) changed_partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// bf16 mode: distances with their error bounds.  Lane q of a column's 16
// lanes takes groups q, q+16, ...  The provisional label is the group with the
// smallest distance; every group whose distance interval [d - 2E, d + 2E] reaches
// below the smallest upper end is a candidate.  A column with more than one
// candidate goes on the refinement list (with up to kMaxCand candidates, or all
// groups) and its label is decided there; the others count their changes here.
__global__ __launch_bounds__(256) void k_dist_argmin_bounded(
    const float* __restrict__ part, const float* __restrict__ ynorm_part, int nslices, int64_t n,
    int c, int kpad, float eps_rel, const double* __restrict__ cnorm,
    const int32_t* __restrict__ old_labels, int32_t* __restrict__ new_labels,
    double* __restrict__ changed_partial, int* __restrict__ counters, int32_t* __restrict__ list,
    int32_t* __restrict__ cand) {
    __shared__ double sh[4];
    const int q = threadIdx.x & 15;
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool live = j < n;
    double ynorm = 0.0;
    if (live)
        for (int s = 0; s < nslices; ++s) ynorm += (double)ynorm_part[(int64_t)s * n + j];
    const double ylen = sqrt(ynorm);
    // pass 1: best distance and the smallest upper bound
    double bestd = INFINITY, upper = INFINITY;
    int bestk = INT_MAX;
    if (live)
        for (int k = q; k < c; k += 16) {
            double dot = 0.0;
            for (int s = 0; s < nslices; ++s) dot += (double)part[((int64_t)s * n + j) * kpad + k];
            const double dist = cnorm[k] - 2.0 * dot;
            const double e = 2.0 * eps_rel * sqrt(cnorm[k]) * ylen;
            if (dist < bestd) { bestd = dist; bestk = k; }
            upper = fmin(upper, dist + e);
        }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        const double od = __shfl_xor(bestd, o, 16);
        const int ok = __shfl_xor(bestk, o, 16);
        if (od < bestd || (od == bestd && ok < bestk)) { bestd = od; bestk = ok; }
        upper = fmin(upper, __shfl_xor(upper, o, 16));
    }
    // pass 2: candidates (lower end below the smallest upper end)
    unsigned long long mine = 0;  // bit t: group q + 16 t is a candidate (first 64 per lane)
    int ncand = 0;
    if (live)
        for (int k = q, t = 0; k < c; k += 16, ++t) {
            double dot = 0.0;
            for (int s = 0; s < nslices; ++s) dot += (double)part[((int64_t)s * n + j) * kpad + k];
            const double dist = cnorm[k] - 2.0 * dot;
            const double e = 2.0 * eps_rel * sqrt(cnorm[k]) * ylen;
            if (dist - e <= upper) { ++ncand; if (t < 64) mine |= 1ull << t; }
        }
    int total = ncand;
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) total += __shfl_xor(total, o, 16);
    double changed = 0.0;
    const int lab = bestk == INT_MAX ? 0 : bestk;
    if (live && total <= 1) {
        if (q == 0) {
            new_labels[j] = lab;
            changed = old_labels[j] != lab ? 1.0 : 0.0;
        }
    } else if (live) {
        // candidate list in increasing group order: rank = candidates of lower groups
        int slot = 0;
        if (q == 0) slot = atomicAdd(&counters[0], 1);
        slot = __shfl(slot, (threadIdx.x & 63) & ~15);
        if (q == 0) { list[slot] = (int32_t)j; new_labels[j] = lab; }
        int32_t* cj = cand + (int64_t)j * kMaxCand;
        if (total > kMaxCand) {
            if (q == 0) cj[0] = -1;          // refine against every group
        } else {
            // groups in increasing order: walk k = 0..c-1, each owned by lane k % 16
            int before = 0;                  // candidates of this lane's groups already placed
            for (int k0 = 0; k0 < c; k0 += 16) {
                const int t = k0 / 16;
                const bool is = (q + k0 < c) && t < 64 && ((mine >> t) & 1ull);
                const unsigned long long bal = __ballot(is);
                const int sub = (threadIdx.x & 63) & ~15;         // this column's 16 lanes
                const unsigned long long grp = (bal >> sub) & 0xFFFFull;
                if (is) cj[before + __popcll(grp & ((1ull << q) - 1ull))] = k0 + q;
                before += __popcll(grp);
            }
            if (q == 0 && total < kMaxCand) cj[total] = -2;   // end marker
        }
    }
    changed = wave_sum_d(changed);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = changed;
    __syncthreads();
    if (threadIdx.x == 0) changed_partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Same decisions as k_dist_argmin_bounded for c <= 16 T, in one pass over the
// partial dot products: a lane keeps the distances and bounds of its T groups in
// registers (the slices are summed in the same order, so every value is
// bitwise the same).
template <int T>
__global__ __launch_bounds__(256) void k_dist_argmin_bounded_r(
    const float* __restrict__ part, const float* __restrict__ ynorm_part, int nslices, int64_t n,
    int c, int kpad, float eps_rel, const double* __restrict__ cnorm,
    const int32_t* __restrict__ old_labels, int32_t* __restrict__ new_labels,
    double* __restrict__ changed_partial, int* __restrict__ counters, int32_t* __restrict__ list,
    int32_t* __restrict__ cand) {
    __shared__ double sh[4];
    const int q = threadIdx.x & 15;
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool live = j < n;
    double ynorm = 0.0;
    double dot[T];
    sum_slices<T, true>(part, ynorm_part, live ? nslices : 0, n, j, c, kpad, q, dot, ynorm);
    const double ylen = sqrt(ynorm);
    double dist[T], err[T];
    double bestd = INFINITY, upper = INFINITY;
    int bestk = INT_MAX;
    double cnv[T];   // loaded unconditionally (clamped), used only below c
#pragma unroll
    for (int t = 0; t < T; ++t) cnv[t] = cnorm[q + 16 * t < c ? q + 16 * t : c - 1];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int k = q + 16 * t;
        dist[t] = INFINITY;
        err[t] = 0.0;
        if (live && k < c) {
            const double cn = cnv[t];
            dist[t] = cn - 2.0 * dot[t];
            err[t] = 2.0 * eps_rel * sqrt(cn) * ylen;
            if (dist[t] < bestd) { bestd = dist[t]; bestk = k; }
            upper = fmin(upper, dist[t] + err[t]);
        }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        const double od = __shfl_xor(bestd, o, 16);
        const int ok = __shfl_xor(bestk, o, 16);
        if (od < bestd || (od == bestd && ok < bestk)) { bestd = od; bestk = ok; }
        upper = fmin(upper, __shfl_xor(upper, o, 16));
    }
    unsigned mine = 0;   // bit t: group q + 16 t is a candidate
    int ncand = 0;
#pragma unroll
    for (int t = 0; t < T; ++t)
        if (live && q + 16 * t < c && dist[t] - err[t] <= upper) { ++ncand; mine |= 1u << t; }
    int total = ncand;
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) total += __shfl_xor(total, o, 16);
    double changed = 0.0;
    const int lab = bestk == INT_MAX ? 0 : bestk;
    if (live && total <= 1) {
        if (q == 0) {
            new_labels[j] = lab;
            changed = old_labels[j] != lab ? 1.0 : 0.0;
        }
    } else if (live) {
        int slot = 0;
        if (q == 0) slot = atomicAdd(&counters[0], 1);
        slot = __shfl(slot, (threadIdx.x & 63) & ~15);
        if (q == 0) { list[slot] = (int32_t)j; new_labels[j] = lab; }
        int32_t* cj = cand + (int64_t)j * kMaxCand;
        if (total > kMaxCand) {
            if (q == 0) cj[0] = -1;          // refine against every group
        } else {
            int before = 0;                  // candidates of lower groups already placed
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const bool is = (mine >> t) & 1u;
                const unsigned long long bal = __ballot(is);
                const int sub = (threadIdx.x & 63) & ~15;
                const unsigned long long grp = (bal >> sub) & 0xFFFFull;
                if (is) cj[before + __popcll(grp & ((1ull << q) - 1ull))] = 16 * t + q;
                before += __popcll(grp);
            }
            if (q == 0 && total < kMaxCand) cj[total] = -2;   // end marker
        }
    }
    changed = wave_sum_d(changed);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = changed;
    __syncthreads();
    if (threadIdx.x == 0) changed_partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// The refinement list, one item per workgroup of kRefineThreads at a time: the
// exact squared distances (double differences of the FP32 values) of the column
// to its candidates -- or, when it had more than kMaxCand, to every group, eight
// at a time -- each thread taking rows tid, tid + kRefineThreads, ... (four rows
// per step, all candidates' loads issued together), reduced over waves in wave
// order; the smallest distance (lowest group on ties) gives the label.
constexpr int kRefineSlots = 256;
constexpr int kRefineThreads = 1024;
constexpr int kRefineRows = 4;   // rows per thread and step, all loads issued together

__global__ __launch_bounds__(kRefineThreads) void k_refine(const float* __restrict__ C, int64_t d,
                                                           int c, const float* __restrict__ Y,
                                                           int64_t ldy,
                                                           const int* __restrict__ counters,
                                                           const int32_t* __restrict__ list,
                                                           const int32_t* __restrict__ cand,
                                                           const int32_t* __restrict__ old_labels,
                                                           int32_t* __restrict__ new_labels,
                                                           int* __restrict__ changed_count) {
    constexpr int NW = kRefineThreads / 64;
    __shared__ double sh[NW][kMaxCand];
    static_assert(kMaxCand == 8, "candidate rows are read as two int4");
    const int count = counters[0];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int item = blockIdx.x; item < count; item += gridDim.x) {
        const int64_t j = list[item];
        const int4* row = reinterpret_cast<const int4*>(cand + j * kMaxCand);
        const int4 c0 = row[0], c1 = row[1];
        const int cv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
        const bool every = cv[0] == -1;
        int ncand = 0;   // candidates up to the first end marker
        if (!every) {
            bool live = true;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                live = live && cv[u] >= 0 && cv[u] < c;
                ncand += live ? 1 : 0;
            }
        }
        const float* y = Y + j * ldy;
        double best = INFINITY;
        int bestk = INT_MAX;
        for (int k0 = 0; k0 < (every ? c : ncand); k0 += 8) {
            int ks[8];
            const int nk = every ? min(8, c - k0) : ncand;
#pragma unroll
            for (int u = 0; u < 8; ++u) ks[u] = every ? min(k0 + u, c - 1) : cv[u < ncand ? u : 0];
            double acc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] = 0.0;
            for (int64_t i = threadIdx.x; i < d; i += kRefineRows * kRefineThreads) {
                // rows i + r kRefineThreads; those past the column's end are clamped
                // into it and contribute zero
                float yv[kRefineRows], cv2[kRefineRows][8];
#pragma unroll
                for (int r = 0; r < kRefineRows; ++r) {
                    const int64_t ii = i + r * kRefineThreads < d ? i + r * kRefineThreads : i;
                    yv[r] = y[ii];
#pragma unroll
                    for (int u = 0; u < 8; ++u) cv2[r][u] = C[(int64_t)ks[u] * d + ii];
                }
#pragma unroll
                for (int r = 0; r < kRefineRows; ++r) {
                    const bool in = i + r * kRefineThreads < d;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const double e = in ? (double)yv[r] - (double)cv2[r][u] : 0.0;
                        acc[u] += e * e;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] = wave_sum_d(acc[u]);
            __syncthreads();   // the previous round's reads of sh are done
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) sh[wave][u] = acc[u];
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int u = 0; u < nk; ++u) {
                    double s = 0.0;
                    for (int w = 0; w < NW; ++w) s += sh[w][u];
                    const int k = every ? k0 + u : cv[u];
                    if (s < best || (s == best && k < bestk)) {
                        best = s;
                        bestk = k;
                    }
                }
            }
            if (!every) break;
        }
        if (threadIdx.x == 0) {
            const int lab = bestk == INT_MAX ? 0 : bestk;
            new_labels[j] = lab;
            if (old_labels[j] != lab) atomicAdd(changed_count, 1);
        }
        __syncthreads();   // sh is reused by the next item
    }
}

// ---- bounded mode with at most 16 groups: FP64 dot products on the vector units
//
// Every product of two FP32 values is exact in FP64, so C_k . Y_j accumulated in
// FP64 carries a relative error of about (K + 16) 2^-53 of sum |c_i y_i| (K rows
// summed per lane): the labels are those of the FP64 distances, as the
// refinement's are, and nothing needs refining.  At c <= 16 the FP64 FMAs stay
// below the time of reading Y once.
//
// A workgroup is 16 lane groups of 16 lanes; group q owns G adjacent columns and
// the workgroup one slice of rows, whose centroid rows it first copies to LDS.
// Lane r of a group holds rows 4r..4r+3 of every 64-row step (16 lanes read 256
// contiguous bytes of a column), loads the next step's rows of its G columns
// before it multiplies the current ones with the centroids from LDS, and keeps
// G x NC FP64 sums; a 16-lane butterfly ends the slice and the per-slice sums go
// to part[slice][column][group].  The workgroups of column block 0 also leave the
// slice's share of ||C_k||^2.
constexpr int kF64MaxC = 16;
constexpr int kF64Lanes = 16;                 // lanes per column group
constexpr int kF64Groups = 256 / kF64Lanes;     // column groups per workgroup
constexpr int kF64Step = 4 * kF64Lanes;         // rows per step of a lane group

// Columns per lane group: at most 6, and G x NC sums of at most 24 doubles.
constexpr int f64_cols(int nc) { return 24 / nc < 1 ? 1 : (24 / nc > 6 ? 6 : 24 / nc); }
// Steps of Y in flight per lane: the current one and kF64Ahead - 1 ahead.
constexpr int kF64Ahead = 3;
// Longest slice: its centroid rows take at most 40 KB of LDS (whole 64-row steps,
// at most 2048 rows).
constexpr int f64_max_rows(int nc) {
    return (40960 / (4 * nc)) / 64 * 64 < 2048 ? (40960 / (4 * nc)) / 64 * 64 : 2048;
}

// Rows rw..rw+3 of column p (VEC: p + rw 16-byte aligned).  FULL: all four rows are
// below lim.  Otherwise rows at or past lim read row lim - 1 and become zero.
template <bool VEC, bool FULL>
__device__ inline float4 load_rows4(const float* __restrict__ p, int64_t rw, int64_t lim) {
    if (VEC) {
        const bool ok = FULL || rw < lim;   // lim is a multiple of 4 here
        float4 v = *reinterpret_cast<const float4*>(p + (ok ? rw : lim - 4));
        if (!ok) v = make_float4(0.f, 0.f, 0.f, 0.f);
        return v;
    }
    float x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool ok = FULL || rw + e < lim;
        x[e] = p[ok ? rw + e : lim - 1];
        if (!ok) x[e] = 0.f;
    }
    return make_float4(x[0], x[1], x[2], x[3]);
}

template <int G, bool VEC, bool FULL>
__device__ inline void f64_load(const float* const (&yc)[G], int64_t rw, int64_t lim, float4 (&y)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) y[g] = load_rows4<VEC, FULL>(yc[g], rw, lim);
}

// acc[g][k] += rows rl..rl+3 of column g times the same rows of centroid k (LDS,
// rows of centroid k at sC[k * R / 4 ...]).
template <int NC, int G, int R>
__device__ inline void f64_fma(const float4 (&y)[G], const float4* sC, int rl, double (&acc)[G][NC]) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const float4 cv = sC[k * (R / 4) + (rl >> 2)];
        const double c0 = cv.x, c1 = cv.y, c2 = cv.z, c3 = cv.w;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double a = acc[g][k];
            a = fma((double)y[g].x, c0, a);
            a = fma((double)y[g].y, c1, a);
            a = fma((double)y[g].z, c2, a);
            a = fma((double)y[g].w, c3, a);
            acc[g][k] = a;
        }
    }
}

template <int NC, bool VEC>
__global__ __launch_bounds__(256) void k_dist_f64(const float* __restrict__ C, int64_t d,
                                                  const float* __restrict__ Y, int64_t ldy, int64_t n,
                                                  int slice_rows, double* __restrict__ part,
                                                  double* __restrict__ cn_part,
                                                  int* __restrict__ counters) {
    constexpr int G = f64_cols(NC);
    constexpr int R = f64_max_rows(NC);   // slice_rows <= R, a multiple of kF64Step
    __shared__ float4 sC[NC * (R / 4)];
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 4)
        counters[threadIdx.x] = 0;   // no refinement list in this mode
    const int r = threadIdx.x & (kF64Lanes - 1);
    const int64_t j0 = (int64_t)blockIdx.x * (kF64Groups * G) + (int64_t)(threadIdx.x / kF64Lanes) * G;
    const int64_t r0 = (int64_t)blockIdx.y * slice_rows;
    const int64_t r1 = r0 + slice_rows < d ? r0 + slice_rows : d;
    const int nfull = (int)((r1 - r0) / kF64Step);              // whole steps
    const int nsteps = (int)((r1 - r0 + kF64Step - 1) / kF64Step);
    // the slice's centroid rows, zero from row r1 to the end of its last step
    const int nq = nsteps * (kF64Step / 4);
    for (int i = threadIdx.x; i < NC * nq; i += 256) {
        const int k = i / nq, q = i - k * nq;
        sC[k * (R / 4) + q] = load_rows4<VEC, false>(C + (int64_t)k * d, r0 + 4 * q, r1);
    }
    __syncthreads();
    const float* yc[G];   // columns past n read column n - 1 and are not written
#pragma unroll
    for (int g = 0; g < G; ++g) yc[g] = Y + (j0 + g < n ? j0 + g : n - 1) * ldy;
    double acc[G][NC];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[g][k] = 0.0;
    const int rl0 = 4 * r;
    if (nfull > 0) {
        // ring of kF64Ahead steps: step t is multiplied while steps t + 1 ..
        // t + kF64Ahead - 1 are in flight; loads past the last whole step re-read it
        // (in bounds, from cache) so that no load sits under a branch
        constexpr int P = kF64Ahead;
        float4 y[P][G];
#pragma unroll
        for (int p = 0; p + 1 < P; ++p)
            f64_load<G, VEC, true>(yc, r0 + rl0 + (int64_t)(p < nfull ? p : nfull - 1) * kF64Step, r1, y[p]);
        int t = 0;
        for (; t + P <= nfull; t += P) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int nx = t + p + P - 1;
                f64_load<G, VEC, true>(yc, r0 + rl0 + (int64_t)(nx < nfull ? nx : nfull - 1) * kF64Step, r1,
                                       y[(p + P - 1) % P]);
                // keep the loads ahead of this step's multiplies (the scheduler would
                // otherwise sink them below, leaving nothing in flight)
                __builtin_amdgcn_sched_barrier(0);
                f64_fma<NC, G, R>(y[p], sC, rl0 + (t + p) * kF64Step, acc);
            }
        }
        // fewer than P steps left, already loaded into y[0 ..]
#pragma unroll
        for (int p = 0; p + 1 < P; ++p)
            if (t + p < nfull) f64_fma<NC, G, R>(y[p], sC, rl0 + (t + p) * kF64Step, acc);
    }
    if (nfull < nsteps) {   // ragged last step: rows from r1 on read as zero
        float4 y[G];
        f64_load<G, VEC, false>(yc, r0 + rl0 + (int64_t)nfull * kF64Step, r1, y);
        f64_fma<NC, G, R>(y, sC, rl0 + nfull * kF64Step, acc);
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int o = kF64Lanes / 2; o > 0; o >>= 1) acc[g][k] += __shfl_xor(acc[g][k], o, kF64Lanes);
    // every lane of the group now holds the same sums; lane r writes group r
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double v = acc[g][0];
#pragma unroll
        for (int k = 1; k < NC; ++k)
            if (r == k) v = acc[g][k];
        if (r < NC && j0 + g < n) part[((int64_t)blockIdx.y * n + j0 + g) * NC + r] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x < 64) {   // this slice's share of ||C_k||^2
        const int lane = threadIdx.x;
#pragma unroll 1
        for (int k = 0; k < NC; ++k) {
            double a = 0.0;
            for (int q = lane; q < nq; q += 64) {
                const float4 v = sC[k * (R / 4) + q];
                a = fma((double)v.x, (double)v.x, a);
                a = fma((double)v.y, (double)v.y, a);
                a = fma((double)v.z, (double)v.z, a);
                a = fma((double)v.w, (double)v.w, a);
            }
            a = wave_sum_d(a);
            if (lane == 0) cn_part[(int64_t)blockIdx.y * NC + k] = a;
        }
    }
}

// One thread per column: slices summed in order, distance ||C_k||^2 - 2 C_k . Y_j
// in FP64, smallest first (lowest group on ties); block 0 also stores ||C_k||^2.
template <int NC>
__global__ __launch_bounds__(256) void k_argmin_f64(const double* __restrict__ part,
                                                    const double* __restrict__ cn_part, int nslices,
                                                    int64_t n, double* __restrict__ cnorm,
                                                    const int32_t* __restrict__ old_labels,
                                                    int32_t* __restrict__ new_labels,
                                                    double* __restrict__ changed_partial) {
    __shared__ double scn[NC];
    __shared__ double sh[4];
    if (threadIdx.x < NC) {
        double a = 0.0;
        for (int s = 0; s < nslices; ++s) a += cn_part[(int64_t)s * NC + threadIdx.x];
        scn[threadIdx.x] = a;
        if (blockIdx.x == 0) cnorm[threadIdx.x] = a;
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = j < n;
    const int64_t jj = live ? j : n - 1;
    double dot[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) dot[k] = 0.0;
#pragma unroll 4
    for (int s = 0; s < nslices; ++s) {
        const double* p = part + ((int64_t)s * n + jj) * NC;
#pragma unroll
        for (int k = 0; k < NC; ++k) dot[k] += p[k];
    }
    double bestd = INFINITY;
    int bestk = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const double dist = scn[k] - 2.0 * dot[k];
        if (dist < bestd) { bestd = dist; bestk = k; }
    }
    double changed = 0.0;
    if (live) {
        new_labels[j] = bestk;
        changed = old_labels[j] != bestk ? 1.0 : 0.0;
    }
    changed = wave_sum_d(changed);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = changed;
    __syncthreads();
    if (threadIdx.x == 0) changed_partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}


struct DistPlan {
    int kpad, ntiles, nkc, slices, slice_rows;
};

// Staged tile (dist_tile): 128 columns per workgroup, slices chosen for at
// least 1024 workgroups.
DistPlan plan_f32(int64_t d, int64_t n, int c) {
    DistPlan p;
    p.kpad = (c + 15) / 16 * 16;
    p.ntiles = (int)((n + kJT - 1) / kJT);
    p.nkc = (p.kpad + kKC - 1) / kKC;
    const int64_t per = (int64_t)p.ntiles * p.nkc;
    int64_t want = (1024 + per - 1) / per;           // aim at >= 1024 workgroups
    const int64_t max_slices = (d + kRT - 1) / kRT;
    if (want > max_slices) want = max_slices;
    if (want > 64) want = 64;
    if (want < 1) want = 1;
    int64_t rows = (d + want - 1) / want;
    rows = (rows + kRT - 1) / kRT * kRT;
    p.slice_rows = (int)rows;
    p.slices = (int)((d + rows - 1) / rows);
    return p;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

// Direct tile: kJD columns per workgroup, one or two workgroups per CU.  The slice count
// minimises the time in units of one stage of every CU: (rounds of workgroups) x
// (stages per slice), plus the partial sums each slice writes and the argmin
// reads back (2 n kpad floats against the CUs' kJD x 32 floats per stage).
DistPlan plan_direct(int64_t d, int64_t n, int c) {
    DistPlan p;
    p.kpad = (c + 15) / 16 * 16;
    p.ntiles = (int)((n + kJD - 1) / kJD);
    p.nkc = (p.kpad + kKC - 1) / kKC;
    const int64_t per = (int64_t)p.ntiles * p.nkc;
    const int64_t slots = (int64_t)device_cus() * direct_wgs_per_cu(std::min(p.kpad / 16, kKC / 16));
    const int64_t stages = (d + kRT - 1) / kRT;
    const double slice_cost = 2.0 * (double)n * p.kpad / ((double)slots * kJD * kRT);
    int64_t best = 1;
    double best_cost = 1e300;
    for (int64_t sl = 1; sl <= 64 && sl <= stages; ++sl) {
        const double cost = (double)(((per * sl + slots - 1) / slots) * ((stages + sl - 1) / sl)) +
                            slice_cost * (double)sl;
        if (cost < best_cost) { best_cost = cost; best = sl; }
    }
    const int64_t rows = (stages + best - 1) / best * kRT;
    p.slice_rows = (int)rows;
    p.slices = (int)((d + rows - 1) / rows);
    return p;
}

// FP64 tile: 16 G columns per workgroup; row slices of whole 64-row steps, at most
// f64_max_rows(c) rows, as many as fill the last round of the workgroups the CUs
// hold at once (per_cu each).
struct F64Plan {
    int ncb, slices, slice_rows;
};

F64Plan plan_f64(int64_t d, int64_t n, int c, int per_cu) {
    F64Plan p;
    const int64_t cols = kF64Groups * (int64_t)f64_cols(c);
    p.ncb = (int)((n + cols - 1) / cols);
    const int64_t steps = (d + kF64Step - 1) / kF64Step;
    const int64_t max_steps = f64_max_rows(c) / kF64Step;
    const int64_t sl_min = (steps + max_steps - 1) / max_steps;
    const int64_t round = (int64_t)device_cus() * per_cu;
    const int64_t rounds = (p.ncb * sl_min + round - 1) / round;
    int64_t sl = std::max<int64_t>(sl_min, rounds * round / p.ncb);
    sl = std::min<int64_t>(sl, steps);
    const int64_t rows = (steps + sl - 1) / sl * kF64Step;
    p.slice_rows = (int)rows;
    p.slices = (int)((d + rows - 1) / rows);
    return p;
}

// Upper bound of plan_f64(d, n, c, per_cu).slices for every per_cu <= 8.
int64_t f64_max_slices(int64_t d, int64_t n, int c) {
    const int64_t cols = kF64Groups * (int64_t)f64_cols(c);
    const int64_t ncb = (n + cols - 1) / cols;
    const int64_t steps = (d + kF64Step - 1) / kF64Step;
    const int64_t max_steps = f64_max_rows(c) / kF64Step;
    const int64_t sl_min = (steps + max_steps - 1) / max_steps;
    return std::min<int64_t>(steps, sl_min + ((int64_t)device_cus() * 8 + ncb - 1) / ncb);
}

// Workgroups of one FP64 tile instance a CU holds at once (from its register use;
// asked once per instance).
template <int NC, bool VEC>
int f64_blocks_per_cu() {
    static const int v = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_dist_f64<NC, VEC>, 256, 0) !=
                hipSuccess || nb < 1)
            nb = 2;
        return std::min(nb, 8);
    }();
    return v;
}

// Bounded mode: at most 16 groups the FP64 tile; at most 32 the FP32 MFMA tile
// with bounds (few MFMAs, no split work); above that the split-bf16 tiles.
constexpr int kF32BoundedMaxC = 32;

bool use_direct(int64_t d, int c, const float* Y, int64_t ldy, bool bf16) {
    return bf16 && c > kF32BoundedMaxC && d % 4 == 0 && ldy % 4 == 0 &&
           reinterpret_cast<uintptr_t>(Y) % 16 == 0;
}

}  // namespace

// Workspace layout (float runs): counters (int x 4, padded to 256 bytes) |
// refinement list [n] | (16-aligned) candidates [n][kMaxCand] | (256-aligned)
// split centroids [kpad][ldq] x 16
// bytes, ldq = ceil(d / 32) * 8 | (256-aligned) partial dots [slices][n][kpad] |
// column norm partials [slices][n], sized for the larger slice count of the two
// tile plans.
int64_t split_ldq(int64_t d) { return (d + kRT - 1) / kRT * (kRT / 4); }

struct WorkLayout {
    int* counters;
    int32_t* list;
    int32_t* cand;
    uint4* csp;
    float* part;
    float* ynorm;
};

inline uintptr_t align_up(uintptr_t v, uintptr_t a) { return (v + a - 1) & ~(a - 1); }

WorkLayout work_layout(void* work, int64_t d, int64_t n, int c, int slices) {
    WorkLayout w;
    const uintptr_t base = (uintptr_t)work;
    w.counters = (int*)base;
    w.list = (int32_t*)(base + 256);
    w.cand = (int32_t*)align_up((uintptr_t)(w.list + n), 16);
    w.csp = (uint4*)align_up((uintptr_t)(w.cand + n * kMaxCand), 256);
    const int kpad = (c + 15) / 16 * 16;
    w.part = (float*)align_up((uintptr_t)(w.csp + (int64_t)kpad * split_ldq(d)), 256);
    w.ynorm = w.part + (size_t)slices * n * kpad;
    return w;
}

// The FP64 tile (c <= 16) puts its double partials [slices][n][c] and the centroid
// norm partials [slices][c] where the float partials start.
template <>
size_t assign_workspace_bytes<float>(int64_t d, int64_t n, int c) {
    const int slices = std::max(plan_f32(d, n, c).slices, plan_direct(d, n, c).slices);
    const WorkLayout w = work_layout(nullptr, d, n, c, slices);
    size_t bytes = (size_t)(uintptr_t)(w.ynorm + (size_t)slices * n);
    if (c <= kF64MaxC) {
        const size_t sf = (size_t)f64_max_slices(d, n, c);
        bytes = std::max(bytes, (size_t)(uintptr_t)w.part + sf * ((size_t)n + 1) * c * sizeof(double));
    }
    return bytes;
}

template <>
size_t assign_workspace_bytes<double>(int64_t d, int64_t n, int c) {
    return (size_t)dots_slices(d, n, c) * (size_t)c * (size_t)n * sizeof(double);
}

template <>
int launch_assign<float>(const float* C, int64_t d, int c, const float* Y, int64_t ldy, int64_t n,
                         double* cnorm, const int32_t* old_labels, int32_t* new_labels,
                         void* work, double* changed_partial, bool bf16, int* changed_extra,
                         hipStream_t st) {
    if (bf16 && c <= kF64MaxC) {
        const WorkLayout w = work_layout(work, d, n, c, 0);
        double* dpart = reinterpret_cast<double*>(w.part);
        const bool vec = (d % 4 == 0) && (ldy % 4 == 0) && (reinterpret_cast<uintptr_t>(Y) % 16 == 0) &&
                         (reinterpret_cast<uintptr_t>(C) % 16 == 0);
        const int ga = (int)((n + 255) / 256);
        switch (c) {
#define RESPCA_F64(NC)                                                                                \
    case NC: {                                                                                        \
        const auto kern = vec ? k_dist_f64<NC, true> : k_dist_f64<NC, false>;                         \
        const F64Plan pf =                                                                            \
            plan_f64(d, n, c, vec ? f64_blocks_per_cu<NC, true>() : f64_blocks_per_cu<NC, false>());  \
        double* cnp = dpart + (size_t)pf.slices * n * c;                                              \
        kern<<<dim3(pf.ncb, pf.slices), 256, 0, st>>>(C, d, Y, ldy, n, pf.slice_rows, dpart, cnp,     \
                                                      w.counters);                                    \
        k_argmin_f64<NC><<<ga, 256, 0, st>>>(dpart, cnp, pf.slices, n, cnorm, old_labels, new_labels, \
                                             changed_partial);                                        \
        break;                                                                                        \
    }
            RESPCA_F64(1) RESPCA_F64(2) RESPCA_F64(3) RESPCA_F64(4) RESPCA_F64(5) RESPCA_F64(6)
            RESPCA_F64(7) RESPCA_F64(8) RESPCA_F64(9) RESPCA_F64(10) RESPCA_F64(11) RESPCA_F64(12)
            RESPCA_F64(13) RESPCA_F64(14) RESPCA_F64(15) RESPCA_F64(16)
#undef RESPCA_F64
        }
        return ga;
    }
    const bool direct = use_direct(d, c, Y, ldy, bf16);
    const DistPlan p = direct ? plan_direct(d, n, c) : plan_f32(d, n, c);
    const WorkLayout w = work_layout(work, d, n, c, p.slices);
    int* counters = w.counters;                       // [0] list length, [1] refined changes
    int32_t* list = w.list;
    int32_t* cand = w.cand;
    uint4* csp = w.csp;
    float* part = w.part;
    float* ynorm = w.ynorm;
    const int64_t ldq = split_ldq(d);
    const dim3 grid(p.ntiles, p.slices, p.nkc);
    const bool vecy = (ldy % 4 == 0) && (reinterpret_cast<uintptr_t>(Y) % 16 == 0);
    const bool vec = vecy && (d % 4 == 0) && (reinterpret_cast<uintptr_t>(C) % 16 == 0);
    const int gb = (int)((n + 15) / 16);
    if (!bf16) {
        if (vec)
            k_dist_mfma<true, false><<<grid, 256, 0, st>>>(C, d, c, p.kpad, Y, ldy, n, p.slice_rows,
                                                           part, ynorm, counters, nullptr, 0);
        else
            k_dist_mfma<false, false><<<grid, 256, 0, st>>>(C, d, c, p.kpad, Y, ldy, n, p.slice_rows,
                                                            part, ynorm, counters, nullptr, 0);
#define RESPCA_ARGMIN_F(TT)                                                                    \
    k_dist_argmin_r<TT><<<gb, 256, 0, st>>>(part, p.slices, n, c, p.kpad, cnorm, old_labels,     \
                                            new_labels, changed_partial)
        if (c <= 16) RESPCA_ARGMIN_F(1);
        else if (c <= 32) RESPCA_ARGMIN_F(2);
        else if (c <= 64) RESPCA_ARGMIN_F(4);
        else if (c <= 128) RESPCA_ARGMIN_F(8);
        else
            k_dist_argmin<<<gb, 256, 0, st>>>(part, p.slices, n, c, p.kpad, cnorm, old_labels,
                                              new_labels, changed_partial);
#undef RESPCA_ARGMIN_F
        return gb;
    }
    // the pre-split centroids replace C in the split tiles, so only Y's layout picks
    // their path; the split pass also leaves the centroid norms
    k_split_centroids<<<p.kpad, 1024, 0, st>>>(
        C, d, c, ldq, (d % 4 == 0) && (reinterpret_cast<uintptr_t>(C) % 16 == 0), csp, cnorm);
    const bool f32b = c <= kF32BoundedMaxC;
    if (f32b) {
        if (vec)
            k_dist_mfma_f32b<true><<<grid, 256, 0, st>>>(C, d, c, p.kpad, Y, ldy, n, p.slice_rows, part,
                                                         ynorm, counters);
        else
            k_dist_mfma_f32b<false><<<grid, 256, 0, st>>>(C, d, c, p.kpad, Y, ldy, n, p.slice_rows, part,
                                                          ynorm, counters);
    } else if (direct) {
        switch (std::min(p.kpad / 16, kKC / 16)) {
#define RESPCA_DIRECT(NB)                                                                            \
    case NB:                                                                                         \
        k_dist_mfma_direct<NB><<<grid, 64 * kDirectWaves, 0, st>>>(d, c, p.kpad, Y, ldy, n,          \
                                                                   p.slice_rows, part, ynorm,        \
                                                                   counters, csp, ldq);              \
        break;
            RESPCA_DIRECT(1) RESPCA_DIRECT(2) RESPCA_DIRECT(3) RESPCA_DIRECT(4)
            RESPCA_DIRECT(5) RESPCA_DIRECT(6) RESPCA_DIRECT(7) RESPCA_DIRECT(8)
#undef RESPCA_DIRECT
        }
    } else
        k_dist_mfma<false, true><<<grid, 256, 0, st>>>(C, d, c, p.kpad, Y, ldy, n, p.slice_rows, part,
                                                       ynorm, counters, csp, ldq);
    // error bound factor (doubled for safety): FP32 accumulation over one slice of
    // rows, plus (split tiles) 3 * 2^-16 per product for the bf16 parts, or (FP32
    // tile) the products' own rounding
    const double acc_err = (p.slice_rows + 2.0) * std::ldexp(1.0, -24);
    const float eps_rel = (float)(2.0 * (f32b ? acc_err : 3.0 * std::ldexp(1.0, -16) + acc_err));
#define RESPCA_ARGMIN_R(TT)                                                                    \
    k_dist_argmin_bounded_r<TT><<<gb, 256, 0, st>>>(part, ynorm, p.slices, n, c, p.kpad, eps_rel,  \
                                                    cnorm, old_labels, new_labels, changed_partial, \
                                                    counters, list, cand)
    if (c <= 16) RESPCA_ARGMIN_R(1);
    else if (c <= 32) RESPCA_ARGMIN_R(2);
    else if (c <= 64) RESPCA_ARGMIN_R(4);
    else if (c <= 128) RESPCA_ARGMIN_R(8);
    else
        k_dist_argmin_bounded<<<gb, 256, 0, st>>>(part, ynorm, p.slices, n, c, p.kpad, eps_rel, cnorm,
                                                  old_labels, new_labels, changed_partial, counters,
                                                  list, cand);
#undef RESPCA_ARGMIN_R
    k_refine<<<kRefineSlots, kRefineThreads, 0, st>>>(C, d, c, Y, ldy, counters, list, cand,
                                                      old_labels, new_labels, counters + 1);
    // refined changes are added to the partial list by the caller via changed_extra
    if (changed_extra) *changed_extra = 1;
    return gb;
}

int* assign_refine_counters(void* work, int64_t, int64_t, int) { return (int*)work; }

template <>
int launch_assign<double>(const double* C, int64_t d, int c, const double* Y, int64_t ldy,
                          int64_t n, double* cnorm, const int32_t* old_labels,
                          int32_t* new_labels, void* work, double* changed_partial, bool,
                          int* changed_extra, hipStream_t st) {
    if (changed_extra) *changed_extra = 0;
    double* part = (double*)work;
    launch_dots<double>(C, d, c, Y, ldy, n, part, st);
    return launch_argmin<double>(part, dots_slices(d, n, c), c, n, cnorm, old_labels, new_labels,
                                 changed_partial, st);
}

}  // namespace respca
