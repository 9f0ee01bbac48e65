// Streaming bandwidth probe: the practical HBM ceiling of a given mix of
// reads and writes on this GPU, with plain or nontemporal loads and stores (the
// l1 sweep on the compact state reads three d x n arrays and writes two; the
// means pass reads two; a copy reads one and writes one).  Used to
// put the streaming kernels' achieved bandwidth beside what the memory system
// delivers for the same mix, not only beside the 8 TB/s peak.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/respca.h"
#include "handle.h"

using namespace respca;

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;   // float4 chunks in flight per thread and array

struct ProbePtrs {
    const float4* in[4];
    float4* out[3];
};

template <int R, int W, bool NT>
__global__ __launch_bounds__(kProbeBlock) void k_stream_mix(ProbePtrs p, int64_t n4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock * kProbeUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kProbeBlock * kProbeUnroll + threadIdx.x; base < n4;
         base += stride) {
        float4 v[R][kProbeUnroll];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u) {
                const int64_t i = base + (int64_t)u * kProbeBlock;
                if (i >= n4) {
                    v[r][u] = make_float4(0.f, 0.f, 0.f, 0.f);
                } else if constexpr (NT) {
                    const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p.in[r] + i));
                    v[r][u] = make_float4(t[0], t[1], t[2], t[3]);
                } else {
                    v[r][u] = p.in[r][i];
                }
            }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kProbeBlock;
            float4 s = v[0][u];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                s.x += v[r][u].x;
                s.y += v[r][u].y;
                s.z += v[r][u].z;
                s.w += v[r][u].w;
            }
            if (i < n4) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const float f = (float)(w + 1);
                    if constexpr (NT)
                        __builtin_nontemporal_store(f4{s.x * f, s.y * f, s.z * f, s.w * f},
                                                    reinterpret_cast<f4*>(p.out[w] + i));
                    else
                        p.out[w][i] = make_float4(s.x * f, s.y * f, s.z * f, s.w * f);
                }
            }
            if (W == 0 && i < n4 && s.x == -1.2345f) p.out[0][i] = s;   // keeps the loads alive
        }
    }
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_fill(float4* a, int64_t n4, float v) {
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
    for (int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n4; i += stride)
        a[i] = make_float4(v, v + 1.f, v + 2.f, v + 3.f);
}

template <int R, int W, bool NT>
void launch_mix(const ProbePtrs& p, int64_t n4, int grid, hipStream_t st) {
    k_stream_mix<R, W, NT><<<grid, kProbeBlock, 0, st>>>(p, n4);
}

using MixFn = void (*)(const ProbePtrs&, int64_t, int, hipStream_t);

template <bool NT>
MixFn mix_fn_t(int r, int w) {
    static const MixFn table[4][4] = {
        {launch_mix<1, 0, NT>, launch_mix<1, 1, NT>, launch_mix<1, 2, NT>, launch_mix<1, 3, NT>},
        {launch_mix<2, 0, NT>, launch_mix<2, 1, NT>, launch_mix<2, 2, NT>, launch_mix<2, 3, NT>},
        {launch_mix<3, 0, NT>, launch_mix<3, 1, NT>, launch_mix<3, 2, NT>, launch_mix<3, 3, NT>},
        {launch_mix<4, 0, NT>, launch_mix<4, 1, NT>, launch_mix<4, 2, NT>, launch_mix<4, 3, NT>}};
    return table[r - 1][w];
}

MixFn mix_fn(int r, int w, bool nt) { return nt ? mix_fn_t<true>(r, w) : mix_fn_t<false>(r, w); }

}  // namespace

extern "C" respca_status respca_bandwidth_probe(respca_handle h, int32_t reads, int32_t writes,
                                                int32_t nontemporal, int64_t bytes_per_array,
                                                int32_t reps, double* gbps, double* ms_per_launch,
                                                void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (reads < 1 || reads > 4 || writes < 0 || writes > 3 || reps < 1 || bytes_per_array < 16 ||
        bytes_per_array % 16 != 0)
        return fail(h, RESPCA_ERR_INVALID,
                    "reads in [1, 4], writes in [0, 3], reps >= 1, bytes a positive multiple of 16");
    CK(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n4 = bytes_per_array / 16;
    const int arrays = reads + (writes > 0 ? writes : 1);
    CKS(ensure(h, h->probe, (size_t)arrays * (size_t)bytes_per_array));
    ProbePtrs p{};
    char* base = (char*)h->probe.p;
    for (int r = 0; r < reads; ++r) p.in[r] = (const float4*)(base + (size_t)r * bytes_per_array);
    for (int w = 0; w < (writes > 0 ? writes : 1); ++w)
        p.out[w] = (float4*)(base + (size_t)(reads + w) * bytes_per_array);
    hipDeviceProp_t prop;
    CK(hipGetDeviceProperties(&prop, h->device));
    const int fill_grid = prop.multiProcessorCount * 8;
    for (int r = 0; r < reads; ++r)
        k_probe_fill<<<fill_grid, kProbeBlock, 0, st>>>((float4*)p.in[r], n4, (float)(r + 1));
    // enough workgroups to keep every CU's waves busy; the rest is grid-stride
    const int64_t need = (n4 + (int64_t)kProbeBlock * kProbeUnroll - 1) / ((int64_t)kProbeBlock * kProbeUnroll);
    const int grid = (int)(need < (int64_t)prop.multiProcessorCount * 16 ? need
                                                                          : (int64_t)prop.multiProcessorCount * 16);
    MixFn fn = mix_fn(reads, writes, nontemporal != 0);
    fn(p, n4, grid, st);   // warm-up
    hipEvent_t a = nullptr, b = nullptr;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
    (void)hipEventRecord(a, st);
    for (int k = 0; k < reps; ++k) fn(p, n4, grid, st);
    (void)hipEventRecord(b, st);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    CK(e);
    CK(hipGetLastError());
    const double per = (double)ms / reps;
    if (ms_per_launch) *ms_per_launch = per;
    if (gbps) *gbps = per > 0 ? (double)(reads + writes) * (double)bytes_per_array / (per * 1e-3) / 1e9 : 0.0;
    return RESPCA_OK;
}
