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
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "kernels.h"

namespace respca {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kJT = 128;     // columns per workgroup
constexpr int kKC = 128;     // groups per workgroup (8 blocks of 16)
constexpr int kRT = 32;      // rows per LDS stage
constexpr int kStride = 36;  // padded LDS stride (floats) of one staged column: conflict-free

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Stage rows [r, r + 32) of `cols` consecutive columns starting at col0 of a
// column-major matrix into LDS (column-major, stride kStride); zero outside.
template <bool VEC>
__device__ inline void stage(float* __restrict__ dst, const float* __restrict__ src, int64_t ld,
                             int64_t col0, int64_t ncols, int64_t r, int64_t rend) {
    const int tid = threadIdx.x;
    if constexpr (VEC) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int col = p * 32 + (tid >> 3);
            const int rr = (tid & 7) * 4;
            const int64_t gj = col0 + col, gi = r + rr;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gj < ncols && gi < rend) v = *reinterpret_cast<const float4*>(src + gj * ld + gi);
            *reinterpret_cast<float4*>(dst + col * kStride + rr) = v;
        }
    } else {
#pragma unroll 4
        for (int e = tid; e < 128 * kRT; e += 256) {
            const int col = e >> 5, rr = e & 31;
            const int64_t gj = col0 + col, gi = r + rr;
            dst[col * kStride + rr] = (gj < ncols && gi < rend) ? src[gj * ld + gi] : 0.f;
        }
    }
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_dist_mfma(const float* __restrict__ C, int64_t d, int c,
                                                   int kpad, const float* __restrict__ Y, int64_t ldy,
                                                   int64_t n, int slice_rows,
                                                   float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) float Ys[kJT * kStride];
    __shared__ __attribute__((aligned(16))) float Cs[kKC * kStride];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int q = lane & 15, g = lane >> 4;
    const int64_t j0 = (int64_t)blockIdx.x * kJT;
    const int s = blockIdx.y;
    const int k0 = blockIdx.z * kKC;
    const int64_t r0 = (int64_t)s * slice_rows;
    const int64_t r1 = r0 + slice_rows < d ? r0 + slice_rows : d;
    const int nkb = (kpad - k0 < kKC ? kpad - k0 : kKC) / 16;

    floatx4 acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int64_t r = r0; r < r1; r += kRT) {
        stage<VEC>(Ys, Y, ldy, j0, n, r, r1);
        stage<VEC>(Cs, C, d, k0, c, r, r1);
        __syncthreads();
        // MFMA step m: lane group g supplies row 8g + m of the stage (same map for both operands)
        float a[2][8];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            const float* p = Ys + (wave * 32 + jb * 16 + q) * kStride + g * 8;
            const float4 u = *reinterpret_cast<const float4*>(p);
            const float4 w = *reinterpret_cast<const float4*>(p + 4);
            a[jb][0] = u.x; a[jb][1] = u.y; a[jb][2] = u.z; a[jb][3] = u.w;
            a[jb][4] = w.x; a[jb][5] = w.y; a[jb][6] = w.z; a[jb][7] = w.w;
        }
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            if (kb < nkb) {
                const float* p = Cs + (kb * 16 + q) * kStride + g * 8;
                const float4 u = *reinterpret_cast<const float4*>(p);
                const float4 w = *reinterpret_cast<const float4*>(p + 4);
                const float b[8] = {u.x, u.y, u.z, u.w, w.x, w.y, w.z, w.w};
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                    for (int m = 0; m < 8; ++m)
                        acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[jb][m], b[m], acc[jb][kb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds D[column 4g + v][group q] of each 16 x 16 tile
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            if (kb >= nkb) continue;
            const int k = k0 + kb * 16 + q;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t j = j0 + wave * 32 + jb * 16 + 4 * g + v;
                if (j < n) part[((int64_t)s * n + j) * kpad + k] = acc[jb][kb][v];
            }
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

struct DistPlan {
    int kpad, ntiles, nkc, slices, slice_rows;
};

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

}  // namespace

template <>
size_t assign_workspace_bytes<float>(int64_t d, int64_t n, int c) {
    const DistPlan p = plan_f32(d, n, c);
    return (size_t)p.slices * (size_t)n * (size_t)p.kpad * sizeof(float);
}

template <>
size_t assign_workspace_bytes<double>(int64_t d, int64_t n, int c) {
    return (size_t)row_blocks(d) * (size_t)c * (size_t)n * sizeof(double);
}

template <>
int launch_assign<float>(const float* C, int64_t d, int c, const float* Y, int64_t ldy, int64_t n,
                         const double* cnorm, const int32_t* old_labels, int32_t* new_labels,
                         void* work, double* changed_partial, hipStream_t st) {
    const DistPlan p = plan_f32(d, n, c);
    float* part = (float*)work;
    const dim3 grid(p.ntiles, p.slices, p.nkc);
    const bool vec = (d % 4 == 0) && (ldy % 4 == 0) && (reinterpret_cast<uintptr_t>(Y) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(C) % 16 == 0);
    if (vec)
        k_dist_mfma<true><<<grid, 256, 0, st>>>(C, d, c, p.kpad, Y, ldy, n, p.slice_rows, part);
    else
        k_dist_mfma<false><<<grid, 256, 0, st>>>(C, d, c, p.kpad, Y, ldy, n, p.slice_rows, part);
    const int gb = (int)((n + 15) / 16);
    k_dist_argmin<<<gb, 256, 0, st>>>(part, p.slices, n, c, p.kpad, cnorm, old_labels, new_labels,
                                      changed_partial);
    return gb;
}

template <>
int launch_assign<double>(const double* C, int64_t d, int c, const double* Y, int64_t ldy,
                          int64_t n, const double* cnorm, const int32_t* old_labels,
                          int32_t* new_labels, void* work, double* changed_partial,
                          hipStream_t st) {
    double* part = (double*)work;
    launch_dots<double>(C, d, c, Y, ldy, n, part, st);
    return launch_argmin<double>(part, row_blocks(d), c, n, cnorm, old_labels, new_labels,
                                 changed_partial, st);
}

int assign_partials(int64_t n) { return (int)((n + 15) / 16); }

}  // namespace respca
