// Column norms of a d x n matrix: the anomaly score of the Sec. 5.3 experiment,
// where the columns of the recovered sparse part S with a large l2 norm mark the
// outlying samples.  One workgroup per column (grid-stride over the columns),
// FP64 sums of the squared stored values: thread t takes rows t, t + 256, ...,
// then the wave sums and the four wave totals in wave order, so every score has
// one fixed summation order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/respca.h"
#include "handle.h"

using namespace respca;

namespace {

constexpr int kNormBlock = 256;

template <typename T>
__global__ __launch_bounds__(kNormBlock) void k_column_norms(const T* __restrict__ S, int64_t lds,
                                                             int64_t d, int64_t n,
                                                             double* __restrict__ out) {
    __shared__ double part[kNormBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        const T* s = S + j * lds;
        double acc = 0.0;
        for (int64_t i = threadIdx.x; i < d; i += kNormBlock) {
            const double v = (double)s[i];
            acc += v * v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        __syncthreads();   // the previous column's totals have been read
        if (lane == 0) part[wave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kNormBlock / 64; ++w) t += part[w];
            out[j] = sqrt(t);
        }
    }
}

}  // namespace

extern "C" respca_status respca_column_norms(respca_handle h, int32_t precision, int64_t d,
                                             int64_t n, const void* S, int64_t lds, double* out,
                                             void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (precision != RESPCA_F64 && precision != RESPCA_F32 && precision != RESPCA_BF16GEMM_F32)
        return fail(h, RESPCA_ERR_INVALID, "precision must be RESPCA_F64, RESPCA_F32 or RESPCA_BF16GEMM_F32");
    if (d < 0 || n < 0 || lds < (d > 1 ? d : 1))
        return fail(h, RESPCA_ERR_INVALID, "column norms: d, n >= 0 and lds >= max(d, 1)");
    if (n == 0) return RESPCA_OK;
    if (!out || (d > 0 && !S)) return fail(h, RESPCA_ERR_INVALID, "column norms: null pointer");
    CK(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    const unsigned grid = (unsigned)(n < 65536 ? n : 65536);
    if (precision == RESPCA_F64)
        k_column_norms<double><<<grid, kNormBlock, 0, st>>>((const double*)S, lds, d, n, out);
    else
        k_column_norms<float><<<grid, kNormBlock, 0, st>>>((const float*)S, lds, d, n, out);
    CK(hipGetLastError());
    return RESPCA_OK;
}
