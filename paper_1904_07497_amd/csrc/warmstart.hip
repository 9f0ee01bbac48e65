// Learned warm start (an addition to the paper's method): column sketches, a
// per-column multilayer perceptron with hand-written forward / backward / Adam
// kernels, and the feature map between them.
//
// Sketch: y_j = R X_j with R[k][i] = +-1/8 taken from bit k of the i-th
// counter-based splitmix64 output (Rademacher projection to 64 dimensions),
// plus ||X_j||.  Network: dims [68, h, h, h, 65], ReLU between layers; inputs
// are the normalised sketch and instance features, outputs the normalised
// sketch of the column's group centroid (64) and a log-threshold (1).
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.h"
#include "warmstart.h"

namespace respca {

namespace {

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t t) {
    uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// One wave per column: 64 projections accumulated per lane over its rows, then
// a butterfly exchange halves the values each lane holds at every stage so that
// lane k ends with the full sum of projection k.  Writes the column's 65 values.
__device__ inline void sketch_column(const float* __restrict__ x, int64_t d, uint64_t seed,
                                     float* __restrict__ yj) {
    const int lane = threadIdx.x & 63;
    float v[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) v[k] = 0.f;
    double nrm = 0.0;
    for (int64_t i = lane; i < d; i += 64) {
        const float xi = x[i];
        const uint64_t bits = splitmix64_at(seed, (uint64_t)i);
        const float p = 0.125f * xi;
#pragma unroll
        for (int k = 0; k < 64; ++k) v[k] += ((bits >> k) & 1ull) ? -p : p;
        nrm += (double)xi * xi;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const bool up = (lane & s) != 0;
#pragma unroll
        for (int k = 0; k < s; ++k) {
            const float send = up ? v[k] : v[k + s];
            const float keep = up ? v[k + s] : v[k];
            v[k] = keep + __shfl_xor(send, s);
        }
    }
    nrm = wave_sum(nrm);
    yj[lane] = v[0];
    if (lane == 0) yj[64] = (float)sqrt(nrm);
}

__global__ __launch_bounds__(256) void k_sketch(const float* __restrict__ X, int64_t ldx, int64_t d,
                                                int64_t n, uint64_t seed, float* __restrict__ Y) {
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    sketch_column(X + j * ldx, d, seed, Y + j * 65);
}

// Instance table of the batched warm start: instance i owns the sketch / feature
// columns [off, off + n) of the concatenation of all instances.
__device__ inline int find_instance(const WarmDesc* __restrict__ D, int batch, int64_t col) {
    int lo = 0, hi = batch;   // D[lo].off <= col < D[hi].off (D[batch].off = total)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (D[mid].off <= col) lo = mid; else hi = mid;
    }
    return lo;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// h[i] = the i-th counter-based splitmix64 output (the signs of sketch row i).
__global__ __launch_bounds__(256) void k_row_hash(uint64_t seed, int64_t rows,
                                                  uint64_t* __restrict__ h) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < rows) h[i] = splitmix64_at(seed, (uint64_t)i);
}

// Batched sketch on the matrix cores: one wave per tile of 16 columns of one
// instance computes Y = R X for all 64 sketch rows with v_mfma_f32_16x16x4f32.
// Lane l (q = l % 16, g = l / 16) feeds column q and, at step e of each 16-row
// chunk, row i0 + 4 g + e: its B value is that entry of X and its A values are
// the signs +-1/8 of sketch rows 16 kb + q for that row (bit 16 kb + q of the row's
// hash); the four lane groups fill the instruction's four K slots.  Column norms
// are summed in double beside the products.
__global__ __launch_bounds__(256) void k_sketch_mfma_b(const WarmDesc* __restrict__ D, int batch,
                                                       int64_t ntiles,
                                                       const uint64_t* __restrict__ hash,
                                                       float* __restrict__ Y) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    int lo = 0, hi = batch;   // D[lo].toff <= tile < D[hi].toff
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (D[mid].toff <= tile) lo = mid; else hi = mid;
    }
    const WarmDesc& w = D[lo];
    const int q = lane & 15, g = lane >> 4;
    const int64_t jl = (tile - w.toff) * 16 + q;   // this lane's column in the instance
    const bool colok = jl < w.n;
    const float* x = w.X + (colok ? jl : 0) * w.ldx;
    const bool vec = (w.ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(w.X) & 15) == 0);
    f32x4 acc[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    double nrm = 0.0;
    // four 16-row steps per pass: their loads are issued together, then the steps
    // are multiplied in row order (the same order as one step at a time)
    constexpr int U = 4;
    for (int64_t i0 = 0; i0 < w.d; i0 += 16 * U) {
        float xv[U][4];
        uint64_t hv[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t r = i0 + 16 * u + 4 * g;
#pragma unroll
            for (int e = 0; e < 4; ++e) { xv[u][e] = 0.f; hv[u][e] = 0; }
            if (vec && r + 4 <= w.d) {
                if (colok) {
                    const float4 t = *reinterpret_cast<const float4*>(x + r);
                    xv[u][0] = t.x; xv[u][1] = t.y; xv[u][2] = t.z; xv[u][3] = t.w;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) hv[u][e] = hash[r + e];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (r + e < w.d) {
                        xv[u][e] = colok ? x[r + e] : 0.f;
                        hv[u][e] = hash[r + e];
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < 4; ++e) nrm += (double)xv[u][e] * (double)xv[u][e];
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    const float a = ((hv[u][e] >> (16 * kb + q)) & 1ull) ? -0.125f : 0.125f;
                    acc[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xv[u][e], acc[kb], 0, 0, 0);
                }
        }
    }
    nrm += __shfl_xor(nrm, 16);
    nrm += __shfl_xor(nrm, 32);
    if (colok) {
        float* yj = Y + (w.off + jl) * 65;
        // lane holds rows 4 g + v of each 16 x 16 output block kb, column q
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int v = 0; v < 4; ++v) yj[16 * kb + 4 * g + v] = acc[kb][v];
        if (g == 0) yj[64] = (float)sqrt(nrm);
    }
}

// sum_j Y[j][64]^2 (= ||X||_F^2) in double, one workgroup.
__global__ __launch_bounds__(256) void k_sketch_total(const float* __restrict__ Y, int64_t n,
                                                      double* __restrict__ out) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double t = Y[j * 65 + 64];
        a += t * t;
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) out[0] = a;
}

// Network inputs of column j: y_j / (s sqrt(d) / 8) (64), log(||X_j|| / (s sqrt(d))),
// log(d) / 8, log(n) / 8, c / 50 with s = ||X||_F / sqrt(d n).
__device__ inline float feature_value(const float* __restrict__ yj, int k, int64_t d, int64_t n,
                                      int64_t c, double total) {
    const double s = sqrt(total / ((double)d * (double)n));
    const double col = s * sqrt((double)d);
    double f;
    if (k < 64) f = (col > 0.0) ? yj[k] / (0.125 * col) : 0.0;
    else if (k == 64) f = log((double)yj[64] / (col > 0.0 ? col : 1.0) + 1e-12);
    else if (k == 65) f = log((double)d) / 8.0;
    else if (k == 66) f = log((double)n) / 8.0;
    else f = (double)c / 50.0;
    return (float)f;
}

__global__ __launch_bounds__(256) void k_features(const float* __restrict__ Y, int64_t d, int64_t n,
                                                  int c, const double* __restrict__ total,
                                                  float* __restrict__ F) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * kWarmIn) return;
    const int64_t j = e / kWarmIn;
    F[e] = feature_value(Y + j * 65, (int)(e % kWarmIn), d, n, c, total[0]);
}

// Batched: one workgroup per instance sums its columns' squared norms (res[2 i]).
__global__ __launch_bounds__(256) void k_sketch_total_b(const WarmDesc* __restrict__ D,
                                                        const float* __restrict__ Y,
                                                        double* __restrict__ res) {
    const WarmDesc& w = D[blockIdx.x];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t j = threadIdx.x; j < w.n; j += 256) {
        const double t = Y[(w.off + j) * 65 + 64];
        a += t * t;
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) res[2 * blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void k_features_b(const WarmDesc* __restrict__ D, int batch,
                                                    int64_t total, const float* __restrict__ Y,
                                                    const double* __restrict__ res,
                                                    float* __restrict__ F) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total * kWarmIn) return;
    const int64_t g = e / kWarmIn;
    const int i = find_instance(D, batch, g);
    const WarmDesc& w = D[i];
    F[e] = feature_value(Y + g * 65, (int)(e % kWarmIn), w.d, w.n, w.c, res[2 * i]);
}

// Batched: one workgroup per instance, mean of its columns' last network output
// (res[2 i + 1]).
__global__ __launch_bounds__(256) void k_pool_last_b(const WarmDesc* __restrict__ D,
                                                     const float* __restrict__ out,
                                                     double* __restrict__ res) {
    const WarmDesc& w = D[blockIdx.x];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t j = threadIdx.x; j < w.n; j += 256) a += out[(w.off + j) * kWarmOut + kWarmOut - 1];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) res[2 * blockIdx.x + 1] = a / (double)w.n;
}

// C(m, n) [+]= sum_k A(m, k) B(k, n) (+ bias[n]) with A(m, k) = A[m*as0 + k*as1],
// B(k, n) = B[k*bs0 + n*bs1], C row-major (ldc).  EPI: 0 none, 1 ReLU, 2 multiply by
// (mask(m, n) > 0) with the mask laid out like C.  64 x 64 tiles, 16-deep K steps
// through LDS, 4 x 4 outputs per thread.
template <bool BIAS, int EPI, bool ACCUM>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              int64_t as0, int64_t as1, const float* __restrict__ B,
                                              int64_t bs0, int64_t bs1, const float* __restrict__ bias,
                                              const float* __restrict__ mask, float* __restrict__ C,
                                              int64_t ldc) {
    __shared__ float As[16][64 + 1];
    __shared__ float Bs[16][64 + 1];
    const int tid = threadIdx.x, tm = tid >> 4, tn = tid & 15;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
    // loads run along whichever index is contiguous in memory (uniform choice)
    const bool a_k_contig = as1 == 1, b_k_contig = bs0 == 1;
    for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int e = tid + 256 * p;        // 1024 = 16 x 64
            {
                const int kk = a_k_contig ? (e & 15) : (e >> 6);
                const int mm = a_k_contig ? (e >> 4) : (e & 63);
                const int gm = m0 + mm, gk = k0 + kk;
                As[kk][mm] = (gm < M && gk < K) ? A[(int64_t)gm * as0 + (int64_t)gk * as1] : 0.f;
            }
            {
                const int kk = b_k_contig ? (e & 15) : (e >> 6);
                const int nn = b_k_contig ? (e >> 4) : (e & 63);
                const int gn = n0 + nn, gk = k0 + kk;
                Bs[kk][nn] = (gn < N && gk < K) ? B[(int64_t)gk * bs0 + (int64_t)gn * bs1] : 0.f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) { a[q] = As[kk][tm * 4 + q]; b[q] = Bs[kk][tn * 4 + q]; }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int m = m0 + tm * 4 + x;
        if (m >= M) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int nn = n0 + tn * 4 + y;
            if (nn >= N) continue;
            float v = acc[x][y];
            if (BIAS) v += bias[nn];
            if (EPI == 1) v = v > 0.f ? v : 0.f;
            if (EPI == 2) v = mask[(int64_t)m * ldc + nn] > 0.f ? v : 0.f;
            float* c = C + (int64_t)m * ldc + nn;
            *c = ACCUM ? *c + v : v;
        }
    }
}

// out[n] = sum_m A[m * lda + n] (fixed order), one thread per column.
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const float* __restrict__ A, int64_t lda,
                                                float* __restrict__ out) {
    const int nn = blockIdx.x * 256 + threadIdx.x;
    if (nn >= N) return;
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += A[(int64_t)m * lda + nn];
    out[nn] = (float)s;
}

// dY = 2 w (Y - T) / B (w = 1 except w_last on the last output), loss partials.
__global__ __launch_bounds__(256) void k_loss(int64_t count, int out_dim, int batch, float w_last,
                                              const float* __restrict__ Y, const float* __restrict__ T,
                                              float* __restrict__ dY, double* __restrict__ partial) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
        const float w = (e % out_dim == out_dim - 1) ? w_last : 1.f;
        const float r = Y[e] - T[e];
        dY[e] = 2.f * w * r / (float)batch;
        a += (double)w * r * r;
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) partial[blockIdx.x] = a / batch;
}

__global__ __launch_bounds__(256) void k_adam(int64_t count, float* __restrict__ p,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// mean_j out[j * 65 + 64] in double, one workgroup.
__global__ __launch_bounds__(256) void k_pool_last(const float* __restrict__ out, int64_t n,
                                                   double* __restrict__ res) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) a += out[j * kWarmOut + kWarmOut - 1];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) res[0] = a / (double)n;
}

void gemm(int M, int N, int K, const float* A, int64_t as0, int64_t as1, const float* B, int64_t bs0,
          int64_t bs1, const float* bias, int epi, const float* mask, bool accum, float* C,
          int64_t ldc, hipStream_t st) {
    const dim3 grid((N + 63) / 64, (M + 63) / 64);
    if (bias && epi == 1 && !accum)
        k_gemm<true, 1, false><<<grid, 256, 0, st>>>(M, N, K, A, as0, as1, B, bs0, bs1, bias, mask, C, ldc);
    else if (bias && epi == 0 && !accum)
        k_gemm<true, 0, false><<<grid, 256, 0, st>>>(M, N, K, A, as0, as1, B, bs0, bs1, bias, mask, C, ldc);
    else if (!bias && epi == 2 && !accum)
        k_gemm<false, 2, false><<<grid, 256, 0, st>>>(M, N, K, A, as0, as1, B, bs0, bs1, bias, mask, C, ldc);
    else
        k_gemm<false, 0, false><<<grid, 256, 0, st>>>(M, N, K, A, as0, as1, B, bs0, bs1, bias, mask, C, ldc);
}

}  // namespace

int64_t mlp_param_count(int hidden) {
    const int dims[5] = {kWarmIn, hidden, hidden, hidden, kWarmOut};
    int64_t t = 0;
    for (int l = 0; l < 4; ++l) t += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
    return t;
}

int64_t mlp_act_count(int hidden, int batch) { return (int64_t)batch * (3 * hidden + kWarmOut); }

void launch_sketch(const float* X, int64_t ldx, int64_t d, int64_t n, uint64_t seed, float* Y,
                   hipStream_t st) {
    k_sketch<<<(unsigned)((n + 3) / 4), 256, 0, st>>>(X, ldx, d, n, seed, Y);
}

void launch_features(const float* Y, int64_t d, int64_t n, int c, double* total, float* F,
                     hipStream_t st) {
    k_sketch_total<<<1, 256, 0, st>>>(Y, n, total);
    k_features<<<(unsigned)((n * kWarmIn + 255) / 256), 256, 0, st>>>(Y, d, n, c, total, F);
}

// acts: [a1 (B x h) | a2 (B x h) | a3 (B x h) | y (B x 65)], y is the network output.
// One dense layer of the forward pass on the FP32 matrix cores:
// C[m][n] = act(sum_k A[m][k] W[n][k] + bias[n]) with A row-major (lda = K), W the
// layer's [N][K] row-major weights and C row-major (ldc = N); K % 4 == 0.  A wave
// takes 16 rows and NB blocks of 16 outputs (the grid's y index steps over
// 16 NB-column chunks); per 16-deep chunk of K, lane (q, g) = (lane % 16, lane / 16)
// loads A[row q][k0 + 4g .. +3] and W[col 16b + q][k0 + 4g .. +3] as single
// 16-byte loads and feeds them to four v_mfma_f32_16x16x4f32 steps: step s takes
// k = k0 + 4g + s from lane group g, the same permutation of K on both operands,
// so each output is the whole sum.  Output register v of a block is row 4g + v,
// column q.
template <int NB, bool RELU>
__global__ __launch_bounds__(256) void k_dense_mfma(int64_t M, int N, int K,
                                                    const float* __restrict__ A,
                                                    const float* __restrict__ W,
                                                    const float* __restrict__ bias,
                                                    float* __restrict__ C) {
    const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (m0 >= M) return;
    const int n0 = blockIdx.y * 16 * NB;
    const int64_t ra = m0 + q < M ? m0 + q : M - 1;   // rows past M: loads clamped, not written
    const float* ap = A + ra * K + 4 * g;
    const float* wp[NB];
    bool wok[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int n = n0 + 16 * b + q;
        wok[b] = n < N;
        wp[b] = W + (int64_t)(wok[b] ? n : 0) * K + 4 * g;
    }
    f32x4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        const bool kok = k0 + 4 * g < K;
        const f32x4 z = f32x4{0.f, 0.f, 0.f, 0.f};
        const f32x4 a = kok ? *reinterpret_cast<const f32x4*>(ap + k0) : z;
        f32x4 w[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) w[b] = (kok && wok[b]) ? *reinterpret_cast<const f32x4*>(wp[b] + k0) : z;
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st], w[b][st], acc[b], 0, 0, 0);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int n = n0 + 16 * b + q;
        if (!wok[b]) continue;
        const float bn = bias[n];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t m = m0 + 4 * g + v;
            if (m >= M) continue;
            float y = acc[b][v] + bn;
            if (RELU) y = y > 0.f ? y : 0.f;
            C[m * N + n] = y;
        }
    }
}

template <int NB>
void dense_mfma(int64_t M, int N, int K, const float* A, const float* W, const float* bias, bool relu,
                float* C, hipStream_t st) {
    const dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 16 * NB - 1) / (16 * NB)));
    if (relu) k_dense_mfma<NB, true><<<grid, 256, 0, st>>>(M, N, K, A, W, bias, C);
    else k_dense_mfma<NB, false><<<grid, 256, 0, st>>>(M, N, K, A, W, bias, C);
}

// A layer through the matrix-core kernel (output blocks per wave: the fewest of
// 1, 2, 4, 5, 8, 16 that cover N, at most 16).
void dense(int64_t M, int N, int K, const float* A, const float* W, const float* bias, bool relu,
           float* C, hipStream_t st) {
    const int nb = (N + 15) / 16;
    if (nb <= 1) dense_mfma<1>(M, N, K, A, W, bias, relu, C, st);
    else if (nb <= 2) dense_mfma<2>(M, N, K, A, W, bias, relu, C, st);
    else if (nb <= 4) dense_mfma<4>(M, N, K, A, W, bias, relu, C, st);
    else if (nb <= 5) dense_mfma<5>(M, N, K, A, W, bias, relu, C, st);
    else if (nb <= 8) dense_mfma<8>(M, N, K, A, W, bias, relu, C, st);
    else dense_mfma<16>(M, N, K, A, W, bias, relu, C, st);
}

void launch_mlp_forward(const float* P, int hidden, int batch, const float* x, float* acts,
                        hipStream_t st) {
    const int dims[5] = {kWarmIn, hidden, hidden, hidden, kWarmOut};
    const float* a = x;
    const float* w = P;
    float* out = acts;
    // the matrix-core layers load 16 bytes at a time: every layer's rows and weight
    // blocks are then 16-byte aligned when the three buffers are (widths are
    // multiples of 4); otherwise the LDS-tiled FP32 kernel
    auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    const bool mfma = al16(P) && al16(x) && al16(acts) && hidden % 4 == 0;
    for (int l = 0; l < 4; ++l) {
        const int in = dims[l], o = dims[l + 1];
        const float* b = w + (int64_t)in * o;
        if (mfma) dense(batch, o, in, a, w, b, l < 3, out, st);   // weights [o][in], bias after them
        else gemm(batch, o, in, a, in, 1, w, 1, in, b, l < 3 ? 1 : 0, nullptr, false, out, o, st);
        a = out;
        out += (int64_t)batch * o;
        w = b + o;
    }
}

void launch_mlp_backward(const float* P, int hidden, int batch, const float* x, const float* acts,
                         const float* dy, float* grad, float* scratch, hipStream_t st) {
    const int dims[5] = {kWarmIn, hidden, hidden, hidden, kWarmOut};
    int64_t woff[4], act_off[4];
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) { woff[l] = o; o += (int64_t)dims[l] * dims[l + 1] + dims[l + 1]; }
    act_off[0] = 0;
    for (int l = 1; l < 4; ++l) act_off[l] = act_off[l - 1] + (int64_t)batch * dims[l];
    // scratch holds two B x h buffers for dZ
    float* dz_a = scratch;
    float* dz_b = scratch + (int64_t)batch * hidden;
    const float* dz = dy;
    for (int l = 3; l >= 0; --l) {
        const int in = dims[l], out = dims[l + 1];
        const float* a_in = l == 0 ? x : acts + act_off[l - 1];
        float* gW = grad + woff[l];
        float* gb = gW + (int64_t)in * out;
        // gW (out x in) = dz^T (out x B) * a_in (B x in)
        gemm(out, in, batch, dz, 1, out, a_in, in, 1, nullptr, 0, nullptr, false, gW, in, st);
        k_colsum<<<(out + 255) / 256, 256, 0, st>>>(batch, out, dz, out, gb);
        if (l > 0) {
            // dz_prev (B x in) = (dz (B x out) * W (out x in)) masked by a_in > 0
            float* nxt = (dz == dz_a) ? dz_b : dz_a;
            gemm(batch, in, out, dz, out, 1, P + woff[l], in, 1, nullptr, 2, a_in, false, nxt, in, st);
            dz = nxt;
        }
    }
}

int launch_loss(int batch, const float* y, const float* t, float w_last, float* dy, double* partial,
                hipStream_t st) {
    const int64_t count = (int64_t)batch * kWarmOut;
    int g = (int)((count + 255) / 256);
    if (g > 1024) g = 1024;
    k_loss<<<g, 256, 0, st>>>(count, kWarmOut, batch, w_last, y, t, dy, partial);
    return g;
}

void launch_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr, float b1,
                 float b2, float eps, int step, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    k_adam<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(count, p, g, m, v, lr, b1, b2, eps, c1, c2);
}

void launch_pool_last(const float* out, int64_t n, double* res, hipStream_t st) {
    k_pool_last<<<1, 256, 0, st>>>(out, n, res);
}

void launch_sketch_batched(const WarmDesc* D, int batch, int64_t total, int64_t ntiles,
                           int64_t max_d, uint64_t* hash, uint64_t seed, float* Y, double* res,
                           float* F, hipStream_t st) {
    k_row_hash<<<(unsigned)((max_d + 255) / 256), 256, 0, st>>>(seed, max_d, hash);
    k_sketch_mfma_b<<<(unsigned)((ntiles + 3) / 4), 256, 0, st>>>(D, batch, ntiles, hash, Y);
    k_sketch_total_b<<<batch, 256, 0, st>>>(D, Y, res);
    k_features_b<<<(unsigned)((total * kWarmIn + 255) / 256), 256, 0, st>>>(D, batch, total, Y, res, F);
}

void launch_pool_last_batched(const WarmDesc* D, int batch, const float* out, double* res,
                              hipStream_t st) {
    k_pool_last_b<<<batch, 256, 0, st>>>(D, out, res);
}

}  // namespace respca
