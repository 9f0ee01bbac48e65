// C ABI of the learned warm start: sketch, features, network training kernels
// and the one-call inference that returns initial labels and rho0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/respca.h"
#include "handle.h"
#include "kernels.h"
#include "warmstart.h"

using namespace respca;

namespace {

bool hidden_ok(int32_t hidden) { return hidden >= 1 && hidden <= 4096; }

}  // namespace

extern "C" {

int64_t respca_mlp_param_count(int32_t hidden) { return hidden_ok(hidden) ? mlp_param_count(hidden) : -1; }

int64_t respca_mlp_act_count(int32_t hidden, int32_t batch) {
    return hidden_ok(hidden) && batch > 0 ? mlp_act_count(hidden, batch) : -1;
}

respca_status respca_sketch(respca_handle h, int64_t d, int64_t n, const void* X, int64_t ldx,
                            uint64_t seed, void* Y, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (d < 1 || n < 1 || !X || !Y || ldx < d) return fail(h, RESPCA_ERR_INVALID, "bad sketch arguments");
    CK(hipSetDevice(h->device));
    launch_sketch((const float*)X, ldx, d, n, seed, (float*)Y, (hipStream_t)stream);
    CK(hipGetLastError());
    return RESPCA_OK;
}

respca_status respca_features(respca_handle h, int64_t d, int64_t n, int32_t c, const void* Y,
                              void* F, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (d < 1 || n < 1 || c < 1 || !Y || !F) return fail(h, RESPCA_ERR_INVALID, "bad feature arguments");
    CK(hipSetDevice(h->device));
    CKS(ensure(h, h->wred, 4 * sizeof(double)));
    launch_features((const float*)Y, d, n, c, (double*)h->wred.p, (float*)F, (hipStream_t)stream);
    CK(hipGetLastError());
    return RESPCA_OK;
}

respca_status respca_mlp_forward(respca_handle h, int32_t hidden, const void* params, int32_t batch,
                                 const void* x, void* acts, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (!hidden_ok(hidden) || batch < 1 || !params || !x || !acts)
        return fail(h, RESPCA_ERR_INVALID, "bad forward arguments");
    CK(hipSetDevice(h->device));
    launch_mlp_forward((const float*)params, hidden, batch, (const float*)x, (float*)acts,
                       (hipStream_t)stream);
    CK(hipGetLastError());
    return RESPCA_OK;
}

respca_status respca_mlp_backward(respca_handle h, int32_t hidden, const void* params, int32_t batch,
                                  const void* x, const void* acts, const void* dy, void* grad,
                                  void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (!hidden_ok(hidden) || batch < 1 || !params || !x || !acts || !dy || !grad)
        return fail(h, RESPCA_ERR_INVALID, "bad backward arguments");
    CK(hipSetDevice(h->device));
    CKS(ensure(h, h->wscratch, 2 * (size_t)batch * hidden * sizeof(float)));
    launch_mlp_backward((const float*)params, hidden, batch, (const float*)x, (const float*)acts,
                        (const float*)dy, (float*)grad, (float*)h->wscratch.p, (hipStream_t)stream);
    CK(hipGetLastError());
    return RESPCA_OK;
}

respca_status respca_mlp_loss(respca_handle h, int32_t batch, const void* y, const void* t,
                              float w_last, void* dy, double* loss, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (batch < 1 || !y || !t || !dy) return fail(h, RESPCA_ERR_INVALID, "bad loss arguments");
    CK(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    CKS(ensure(h, h->wred, 1040 * sizeof(double)));
    double* part = (double*)h->wred.p + 8;
    const int g = launch_loss(batch, (const float*)y, (const float*)t, w_last, (float*)dy, part, st);
    if (loss) {
        launch_sum_partials(part, g, 1, (double*)h->wred.p, st);
        CKS(ensure_host(h, 16 * sizeof(double)));
        CK(hipMemcpyAsync(h->hstage, h->wred.p, sizeof(double), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        *loss = h->hstage[0];
    }
    return RESPCA_OK;
}

respca_status respca_mlp_adam(respca_handle h, int64_t count, void* params, const void* grad, void* m,
                              void* v, float lr, float beta1, float beta2, float eps, int32_t step,
                              void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (count < 1 || !params || !grad || !m || !v || step < 1)
        return fail(h, RESPCA_ERR_INVALID, "bad adam arguments");
    CK(hipSetDevice(h->device));
    launch_adam(count, (float*)params, (const float*)grad, (float*)m, (float*)v, lr, beta1, beta2, eps,
                step, (hipStream_t)stream);
    CK(hipGetLastError());
    return RESPCA_OK;
}

respca_status respca_warmstart(respca_handle h, int32_t hidden, const void* params, int64_t d,
                               int64_t n, int32_t c, const void* X, int64_t ldx,
                               uint64_t sketch_seed, uint64_t kmeans_seed, int32_t* init_labels,
                               double* rho0, int32_t* fallback, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (!hidden_ok(hidden) || !params || !X || !init_labels || !rho0 || d < 1 || n < 1 ||
        ldx < d || c < 1 || c > n || c > kMaxGroups || n >= INT32_MAX)
        return fail(h, RESPCA_ERR_INVALID, "bad warm-start arguments");
    CK(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    CKS(ensure(h, h->wsk, (size_t)65 * n * sizeof(float)));
    CKS(ensure(h, h->wfeat, (size_t)kWarmIn * n * sizeof(float)));
    CKS(ensure(h, h->wacts, (size_t)mlp_act_count(hidden, (int)n) * sizeof(float)));
    CKS(ensure(h, h->wred, 1040 * sizeof(double)));
    CKS(ensure(h, h->wcent, (size_t)64 * c * sizeof(float)));
    CKS(ensure_host(h, 16 * sizeof(double)));
    float* Y = (float*)h->wsk.p;
    float* F = (float*)h->wfeat.p;
    float* A = (float*)h->wacts.p;
    double* red = (double*)h->wred.p;
    launch_sketch((const float*)X, ldx, d, n, sketch_seed, Y, st);
    launch_features(Y, d, n, c, red, F, st);
    launch_mlp_forward((const float*)params, hidden, (int)n, F, A, st);
    const float* out = A + (int64_t)3 * n * hidden;      // n x 65
    launch_pool_last(out, n, red + 1, st);
    CK(hipMemcpyAsync(h->hstage, red, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    // read before the K-means below, which reuses the host staging area
    const double total = h->hstage[0], tmean = h->hstage[1];
    // initial groups: K-means of the predicted centroid sketches (column j = out row j, ld 65)
    int steps = 0;
    CKS(kmeans_f32(h, 64, n, c, out, kWarmOut, kmeans_seed, 100, init_labels, (float*)h->wcent.p, st,
                   &steps));
    CK(hipStreamSynchronize(st));
    const double s = std::sqrt(total / ((double)d * (double)n));
    double r = (s > 0.0) ? std::exp(tmean) / s : NAN;
    int fb = 0;
    if (!(r > 0.0) || !std::isfinite(r) || r > 1e10) { r = 1e-4; fb = 1; }
    *rho0 = r;
    if (fallback) *fallback = fb;
    return RESPCA_OK;
}

respca_status respca_warmstart_batched(respca_handle h, int32_t hidden, const void* params,
                                       int32_t batch, const int64_t* d, const int64_t* n,
                                       const int32_t* c, const void* const* X, const int64_t* ldx,
                                       uint64_t sketch_seed, void* embedding, double* rho0,
                                       int32_t* fallback, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    if (!hidden_ok(hidden) || !params || batch < 1 || batch > 1024 || !d || !n || !c || !X || !ldx ||
        !embedding || !rho0)
        return fail(h, RESPCA_ERR_INVALID, "bad batched warm-start arguments");
    int64_t total = 0;
    for (int i = 0; i < batch; ++i) {
        if (!X[i] || d[i] < 1 || n[i] < 1 || ldx[i] < d[i] || c[i] < 1 || c[i] > n[i])
            return fail(h, RESPCA_ERR_INVALID, "bad batched warm-start instance");
        total += n[i];
    }
    if (total >= INT32_MAX / kWarmOut) return fail(h, RESPCA_ERR_UNSUPPORTED, "too many columns");
    CK(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    CKS(ensure(h, h->wsk, (size_t)65 * total * sizeof(float)));
    CKS(ensure(h, h->wfeat, (size_t)kWarmIn * total * sizeof(float)));
    CKS(ensure(h, h->wacts, (size_t)mlp_act_count(hidden, (int)total) * sizeof(float)));
    CKS(ensure(h, h->wred, (size_t)2 * batch * sizeof(double)));
    CKS(ensure(h, h->wdesc, (size_t)batch * sizeof(WarmDesc)));
    const size_t desc_bytes = (size_t)batch * sizeof(WarmDesc);
    CKS(ensure_host(h, std::max(desc_bytes, (size_t)2 * batch * sizeof(double))));
    float* Y = (float*)h->wsk.p;
    float* F = (float*)h->wfeat.p;
    float* A = (float*)h->wacts.p;
    double* red = (double*)h->wred.p;
    // instance table, staged through pinned memory (one launch per stage for all instances)
    WarmDesc* hd = reinterpret_cast<WarmDesc*>(h->hstage);
    int64_t off = 0, toff = 0, max_d = 1;
    for (int i = 0; i < batch; ++i) {
        hd[i] = WarmDesc{(const float*)X[i], ldx[i], d[i], n[i], off, c[i], toff};
        off += n[i];
        toff += (n[i] + 15) / 16;
        max_d = std::max(max_d, d[i]);
    }
    CKS(ensure(h, h->whash, (size_t)max_d * sizeof(uint64_t)));
    const WarmDesc* D = (const WarmDesc*)h->wdesc.p;
    CK(hipMemcpyAsync(h->wdesc.p, hd, desc_bytes, hipMemcpyHostToDevice, st));
    launch_sketch_batched(D, batch, total, toff, max_d, (uint64_t*)h->whash.p, sketch_seed, Y, red, F,
                          st);
    launch_mlp_forward((const float*)params, hidden, (int)total, F, A, st);
    const float* out = A + (int64_t)3 * total * hidden;   // total x 65
    launch_pool_last_batched(D, batch, out, red, st);
    CK(hipMemcpyAsync(embedding, out, (size_t)kWarmOut * total * sizeof(float), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(h->hstage, red, 2 * (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (int i = 0; i < batch; ++i) {
        const double s = std::sqrt(h->hstage[2 * i] / ((double)d[i] * (double)n[i]));
        double r = (s > 0.0) ? std::exp(h->hstage[2 * i + 1]) / s : NAN;
        int fb = 0;
        if (!(r > 0.0) || !std::isfinite(r) || r > 1e10) { r = 1e-4; fb = 1; }
        rho0[i] = r;
        if (fallback) fallback[i] = fb;
    }
    return RESPCA_OK;
}

}  // extern "C"
