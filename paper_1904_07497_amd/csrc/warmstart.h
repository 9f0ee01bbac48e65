// Learned warm start: launchers of the sketch, feature and network kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace respca {

constexpr int kWarmIn = 68;    // 64 sketch coordinates, log column norm, log d, log n, c
constexpr int kWarmOut = 65;   // 64 centroid-sketch coordinates, log threshold

int64_t mlp_param_count(int hidden);
int64_t mlp_act_count(int hidden, int batch);
void launch_sketch(const float* X, int64_t ldx, int64_t d, int64_t n, uint64_t seed, float* Y,
                   hipStream_t st);
void launch_features(const float* Y, int64_t d, int64_t n, int c, double* total, float* F,
                     hipStream_t st);
void launch_mlp_forward(const float* P, int hidden, int batch, const float* x, float* acts,
                        hipStream_t st);
void launch_mlp_backward(const float* P, int hidden, int batch, const float* x, const float* acts,
                         const float* dy, float* grad, float* scratch, hipStream_t st);
int launch_loss(int batch, const float* y, const float* t, float w_last, float* dy, double* partial,
                hipStream_t st);
void launch_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr, float b1,
                 float b2, float eps, int step, hipStream_t st);
void launch_pool_last(const float* out, int64_t n, double* res, hipStream_t st);

// One instance of a batched warm start: its columns are [off, off + n) of the
// concatenated sketch / feature / output arrays (entry batch holds off = total).
struct WarmDesc {
    const float* X;
    int64_t ldx, d, n, off, c;
    int64_t toff;   // first of the instance's ceil(n / 16) sketch tiles
};
// Sketch, squared-norm totals (res[2 i]) and features of every instance's columns;
// `hash` is scratch for max_d row hashes (max_d = the largest d).
void launch_sketch_batched(const WarmDesc* D, int batch, int64_t total, int64_t ntiles,
                           int64_t max_d, uint64_t* hash, uint64_t seed, float* Y, double* res,
                           float* F, hipStream_t st);
// Mean of each instance's last network output (res[2 i + 1]).
void launch_pool_last_batched(const WarmDesc* D, int batch, const float* out, double* res,
                              hipStream_t st);

}  // namespace respca
