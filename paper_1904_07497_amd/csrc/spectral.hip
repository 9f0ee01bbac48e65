// Spectral-clustering p-step (the nonlinear alternative to K-means named at the
// end of Sec. 4.2 and in the Remark closing Sec. 3), as normalised spectral
// clustering: affinity W_ij = exp(-||y_i - y_j||^2 / (2 sigma^2)) (zero
// diagonal), A = D^{-1/2} W D^{-1/2}, the eigenvectors of the c largest
// eigenvalues of A, rows scaled to unit length; the rows are then clustered by
// the K-means machinery of the solver.
//
// GPU design (all FP64 after the load of the columns):
//   - W from the Gram matrix Y^T Y on FP64 MFMA tiles (v_mfma_f64_16x16x4f64) of
//     the upper triangle, the Gaussian of q_i + q_j - 2 G_ij applied in the
//     tile's epilogue and the tile written with its mirror, so the Gram matrix is
//     never stored (the one dense GEMM of the method);
//   - degrees (one wave per row, fixed order); A itself is never formed: a block
//     product A Y is computed as s o (W (s o Y)) with s = D^{-1/2}, the two
//     diagonal scalings folded into the product's load and reduction;
//   - the top-c eigenvectors by Chebyshev-filtered subspace iteration with a
//     block of k = min(n, c + 8) vectors: block products A Y on FP64 MFMA read W
//     once per product, Rayleigh-Ritz in one workgroup (Cholesky of Y^T Y,
//     Jacobi on the k x k projected matrix), two Rayleigh-Ritz passes per filter
//     so the block stays orthonormal to rounding; within a solve each p-step's
//     iteration starts from the previous p-step's Ritz vectors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/respca.h"
#include "handle.h"
#include "kernels.h"
#include "spectral.h"

namespace respca {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kSpBlock = 256;
constexpr int kGramTile = 64;   // output tile of the affinity kernel (64 x 64)
constexpr int kGramK = 16;      // rows of Y per LDS stage

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// q_j = ||Y_j||^2 in double, one wave per column, fixed order; with mean (the
// mean column), also dev[j] = ||Y_j - mean||^2.
template <typename T>
__global__ __launch_bounds__(kSpBlock) void k_sp_colsq(const T* __restrict__ Y, int64_t ldy,
                                                       int64_t d, int64_t n, double* __restrict__ q,
                                                       const double* __restrict__ mean,
                                                       double* __restrict__ dev) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    const T* y = Y + j * ldy;
    double s = 0.0, e = 0.0;
    for (int64_t i = lane; i < d; i += 64) {
        const double v = (double)y[i];
        s += v * v;
        if (mean) {
            const double u = v - mean[i];
            e += u * u;
        }
    }
    s = wsum(s);
    if (lane == 0) q[j] = s;
    if (mean) {
        e = wsum(e);
        if (lane == 0) dev[j] = e;
    }
}

// Column sums of Y over column splits: part[s][i] = sum over the split's columns
// (in order) of Y[i][j]; thread = row i.
template <typename T>
__global__ __launch_bounds__(kSpBlock) void k_sp_rowsum(const T* __restrict__ Y, int64_t ldy,
                                                        int64_t d, int64_t n, int64_t jchunk,
                                                        double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    if (i >= d) return;
    const int64_t jb = (int64_t)blockIdx.y * jchunk;
    const int64_t je = jb + jchunk < n ? jb + jchunk : n;
    double s = 0.0;
    for (int64_t j = jb; j < je; ++j) s += (double)Y[j * ldy + i];
    part[(int64_t)blockIdx.y * d + i] = s;
}

// mean[i] = (sum of the splits' partials, in order) / n.
__global__ __launch_bounds__(kSpBlock) void k_sp_mean(const double* __restrict__ part, int splits,
                                                      int64_t d, int64_t n, double* __restrict__ mean) {
    const int64_t i = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    if (i >= d) return;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[(int64_t)sp * d + i];
    mean[i] = s / (double)n;
}

// out[3] = (1/n) sum_j dev[j] (the squared spread), one workgroup, fixed order.
__global__ __launch_bounds__(kSpBlock) void k_sp_spread(const double* __restrict__ dev, int64_t n,
                                                        double* __restrict__ out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += kSpBlock) s += dev[j];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[3] = (((red[0] + red[1]) + red[2]) + red[3]) / (double)n;
}

// W[i*n + j] = exp(-max(q_i + q_j - 2 G_ij, 0) * inv2s2) for i != j, 0 on the
// diagonal, G = Y^T Y.  One workgroup per 64 x 64 tile of the upper triangle
// (i block = blockIdx.x <= j block = blockIdx.y; the others leave at once); four
// waves of 32 x 32, each 2 x 2 FP64 MFMA blocks of 16 x 16.  The tile's values
// pass through LDS (rows skewed by their index, so reading a column is free of
// bank conflicts) and are written twice, as rows of W and (off the diagonal) as
// rows of the transposed tile, both with 64 consecutive doubles per wave.
template <typename T>
__global__ __launch_bounds__(kSpBlock) void k_sp_affinity(const T* __restrict__ Y, int64_t ldy,
                                                          int64_t d, int64_t n,
                                                          const double* __restrict__ q, double inv2s2,
                                                          double* __restrict__ W) {
    if (blockIdx.x > blockIdx.y) return;   // lower triangle: written by its mirror tile
    // two stages of A and B, rows padded by 16 doubles so that the lanes reading
    // four consecutive rows of a stage fall in different banks; then the tile
    constexpr int kPad = kGramTile + 16;
    __shared__ double smem[2 * 2 * kGramK * kPad];
    static_assert(2 * 2 * kGramK * kPad >= kGramTile * kGramTile, "the tile fits the staging space");
    double (*As)[kGramK][kPad] = reinterpret_cast<double (*)[kGramK][kPad]>(smem);
    double (*Bs)[kGramK][kPad] = reinterpret_cast<double (*)[kGramK][kPad]>(smem + 2 * kGramK * kPad);
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kGramTile;
    const int64_t j0 = (int64_t)blockIdx.y * kGramTile;
    // loader: thread t takes column t/4 of the tile and rows 4 (t%4) .. +3 of the stage
    const int lc = t >> 2;
    const int lr = (t & 3) * 4;
    const int64_t ci = i0 + lc, cj = j0 + lc;
    const T* yi = Y + (ci < n ? ci : 0) * ldy;
    const T* yj = Y + (cj < n ? cj : 0) * ldy;
    const bool vi = ci < n, vj = cj < n;
    double ra[4], rb[4];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = k0 + lr + r;
            ra[r] = (vi && row < d) ? (double)yi[row] : 0.0;
            rb[r] = (vj && row < d) ? (double)yj[row] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            As[buf][lr + r][lc] = ra[r];
            Bs[buf][lr + r][lc] = rb[r];
        }
    };
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int64_t stages = (d + kGramK - 1) / kGramK;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int64_t s = 0; s < stages; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < stages) fetch((s + 1) * kGramK);   // next stage in flight during the MFMAs
#pragma unroll
        for (int kk = 0; kk < kGramK; kk += 4) {
            const int kr = kk + (lane >> 4);
            double a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = As[buf][kr][wi + x * 16 + (lane & 15)];
                b[x] = Bs[buf][kr][wj + x * 16 + (lane & 15)];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        if (s + 1 < stages) stash(buf ^ 1);
        __syncthreads();
    }
    // epilogue: register r of a lane holds row lane / 16 + 4 r, column lane % 16 of
    // each 16 x 16 block (the FP64 MFMA's output order); tile element (mm, nn) goes
    // to smem[mm * 64 + (nn + mm) % 64]
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int mm = wi + x * 16 + (lane >> 4) + 4 * r;
                const int nn = wj + y * 16 + (lane & 15);
                const int64_t i = i0 + mm, j = j0 + nn;
                const double dist = ((i < n) ? q[i] : 0.0) + ((j < n) ? q[j] : 0.0) - 2.0 * acc[x][y][r];
                smem[mm * kGramTile + ((nn + mm) & (kGramTile - 1))] =
                    (i == j) ? 0.0 : exp(-(dist > 0.0 ? dist : 0.0) * inv2s2);
            }
    __syncthreads();
    for (int e = t; e < kGramTile * kGramTile; e += kSpBlock) {
        const int mm = e / kGramTile, nn = e % kGramTile;
        const int64_t i = i0 + mm, j = j0 + nn;
        if (i < n && j < n) W[i * n + j] = smem[mm * kGramTile + ((nn + mm) & (kGramTile - 1))];
    }
    if (blockIdx.x == blockIdx.y) return;
    for (int e = t; e < kGramTile * kGramTile; e += kSpBlock) {
        const int nn = e / kGramTile, mm = e % kGramTile;
        const int64_t i = i0 + mm, j = j0 + nn;
        if (i < n && j < n) W[j * n + i] = smem[mm * kGramTile + ((nn + mm) & (kGramTile - 1))];
    }
}

// s_i = deg_i^{-1/2} (0 for deg_i = 0), deg_i = sum_j W_ij in index order per
// lane, then a butterfly; one wave per row.
__global__ __launch_bounds__(kSpBlock) void k_sp_degree(const double* __restrict__ W, int64_t n,
                                                        double* __restrict__ s) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double* w = W + i * n;
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += 64) acc += w[j];
    acc = wsum(acc);
    if (lane == 0) s[i] = acc > 0.0 ? 1.0 / sqrt(acc) : 0.0;
}

// Block product split over the summation index, P[split][i][q] = sum over j in
// the split's range of A_ij s_j Y[j][q] (A is the affinity W, symmetric: A_ij is
// stored at A[j n + i]; s_j is applied as Y is staged), on FP64 MFMA
// (v_mfma_f64_16x16x4f64): a wave owns 16 rows i and multiplies A[i][j0..j0+3]
// (A operand, lane = row i % 16 and j offset lane / 16: 128 contiguous bytes of A
// per j) by s_j Y[j0..j0+3][16 columns] (B operand, staged in LDS 64 rows at a
// time for the four waves of the workgroup, columns past k zero), NQB blocks of
// 16 columns; sixteen j steps' loads of A are issued before the stage's Y is
// staged and before their MFMAs.
constexpr int kMvRows = 64;   // Y rows staged per LDS pass

template <int NQB>
__global__ __launch_bounds__(kSpBlock) void k_sp_mv_mfma(const double* __restrict__ A, int64_t n,
                                                         const double* __restrict__ Y, int k,
                                                         int64_t jchunk, const double* __restrict__ sj,
                                                         double* __restrict__ P) {
    __shared__ double Ys[kMvRows][16 * NQB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + wave * 16 + (lane & 15);
    const bool live = i < n;
    const int64_t jb = (int64_t)blockIdx.y * jchunk;
    int64_t je = jb + jchunk;
    if (je > n) je = n;
    dbl4 acc[NQB];
#pragma unroll
    for (int x = 0; x < NQB; ++x) acc[x] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int jo = lane >> 4;   // j offset within a step of four
    for (int64_t js = jb; js < je; js += kMvRows) {
        // the stage's loads of A go out before the staging of Y, so the two overlap
        double a[kMvRows / 4];
#pragma unroll
        for (int st = 0; st < kMvRows / 4; ++st) {
            const int64_t j = js + 4 * st + jo;
            a[st] = (live && j < je) ? A[j * n + i] : 0.0;
        }
        for (int e = t; e < kMvRows * 16 * NQB; e += kSpBlock) {
            const int jj = e / (16 * NQB), q = e - jj * (16 * NQB);
            const int64_t j = js + jj;
            Ys[jj][q] = (j < je && q < k) ? sj[j] * Y[j * k + q] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < kMvRows / 4; ++st)
#pragma unroll
            for (int x = 0; x < NQB; ++x)
                acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], Ys[4 * st + jo][16 * x + (lane & 15)],
                                                             acc[x], 0, 0, 0);
        __syncthreads();
    }
    // register r of a lane: row lane / 16 + 4 r of the wave's 16, column lane % 16
#pragma unroll
    for (int x = 0; x < NQB; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + (lane >> 4) + 4 * r;
            const int q = 16 * x + (lane & 15);
            if (row < n && q < k) P[((int64_t)blockIdx.y * n + row) * k + q] = acc[x][r];
        }
}

// Z[i][q] = s_i times the sum over splits (in order) of P[split][i][q].
__global__ __launch_bounds__(kSpBlock) void k_sp_mv_reduce(const double* __restrict__ P, int splits,
                                                           int64_t nk, int k,
                                                           const double* __restrict__ si,
                                                           double* __restrict__ Z) {
    const int64_t e = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    if (e >= nk) return;
    double s = P[e];
    for (int sp = 1; sp < splits; ++sp) s += P[(int64_t)sp * nk + e];
    Z[e] = si[e / k] * s;
}

// Chebyshev step on rows: out = alpha (Z - c0 Y) - beta Yprev.
__global__ __launch_bounds__(kSpBlock) void k_sp_cheb(const double* __restrict__ Z,
                                                      const double* __restrict__ Y,
                                                      const double* __restrict__ Yp, double c0,
                                                      double alpha, double beta, int64_t nk,
                                                      double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    if (e >= nk) return;
    double v = alpha * (Z[e] - c0 * Y[e]);
    if (beta != 0.0) v -= beta * Yp[e];
    out[e] = v;
}

// Partial Gram matrices over row chunks: part[b] = (Y^T Y, Y^T Z) of rows
// [b*rows, (b+1)*rows), k x k each, thread per (p, q) pair.
__global__ __launch_bounds__(kSpBlock) void k_sp_gram(const double* __restrict__ Y,
                                                      const double* __restrict__ Z, int64_t n, int k,
                                                      int64_t rows, double* __restrict__ part) {
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    int64_t r1 = r0 + rows;
    if (r1 > n) r1 = n;
    const int kk = k * k;
    double* out = part + (int64_t)blockIdx.x * 2 * kk;
    for (int pq = threadIdx.x; pq < kk; pq += kSpBlock) {
        const int p = pq / k, q = pq - p * k;
        double g = 0.0, hh = 0.0;
        for (int64_t j = r0; j < r1; ++j) {
            const double yp = Y[j * k + p];
            g += yp * Y[j * k + q];
            hh += yp * Z[j * k + q];
        }
        out[pq] = g;
        out[kk + pq] = hh;
    }
}

// Rayleigh-Ritz on the k x k pair (G, H) in one workgroup: sums the partials
// (in order), G = R^T R (Cholesky), H' = R^{-T} H R^{-1} (symmetrised), Jacobi
// sweeps to diagonalise H' = V Theta V^T, eigenpairs sorted by decreasing value,
// M = R^{-1} V.  out: M (k x k, row-major), theta (k), flag (1.0 if G was not
// positive definite).
constexpr int kSpMaxK = 48;   // eigen block limit (c + 8 with c <= 40)

__global__ __launch_bounds__(kSpBlock) void k_sp_rr(const double* __restrict__ part, int nparts,
                                                    int k, double* __restrict__ M,
                                                    double* __restrict__ theta,
                                                    double* __restrict__ flag) {
    __shared__ double G[kSpMaxK][kSpMaxK + 1];
    __shared__ double H[kSpMaxK][kSpMaxK + 1];
    __shared__ double V[kSpMaxK][kSpMaxK + 1];
    __shared__ double cs[kSpMaxK / 2][2];
    __shared__ int pairs[kSpMaxK];
    __shared__ int bad;
    __shared__ double offsum;
    const int t = threadIdx.x;
    const int kk = k * k;
    for (int pq = t; pq < kk; pq += kSpBlock) {
        double g = 0.0, hh = 0.0;
        for (int b = 0; b < nparts; ++b) {
            g += part[(int64_t)b * 2 * kk + pq];
            hh += part[(int64_t)b * 2 * kk + kk + pq];
        }
        G[pq / k][pq % k] = g;
        H[pq / k][pq % k] = hh;
    }
    if (t == 0) bad = 0;
    __syncthreads();
    // Cholesky, upper factor R in the upper triangle of G (G = R^T R)
    for (int j = 0; j < k; ++j) {
        if (t == 0) {
            double s = G[j][j];
            for (int p = 0; p < j; ++p) s -= G[p][j] * G[p][j];
            if (!(s > 0.0)) {
                bad = 1;
                s = 1e-300;
            }
            G[j][j] = sqrt(s);
        }
        __syncthreads();
        for (int c = j + 1 + t; c < k; c += kSpBlock) {
            double s = G[j][c];
            for (int p = 0; p < j; ++p) s -= G[p][j] * G[p][c];
            G[j][c] = s / G[j][j];
        }
        __syncthreads();
    }
    // V <- R^{-1} (upper triangular), one column per thread
    for (int c = t; c < k; c += kSpBlock) {
        for (int r = k - 1; r >= 0; --r) {
            double s = (r == c) ? 1.0 : 0.0;
            for (int p = r + 1; p <= c; ++p) s -= G[r][p] * V[p][c];
            V[r][c] = (r <= c) ? s / G[r][r] : 0.0;
        }
    }
    __syncthreads();
    // G <- H R^{-1}, then H <- R^{-T} G, symmetrised
    for (int pq = t; pq < kk; pq += kSpBlock) {
        const int p = pq / k, q = pq % k;
        double s = 0.0;
        for (int r = 0; r <= q; ++r) s += H[p][r] * V[r][q];
        G[p][q] = s;
    }
    __syncthreads();
    for (int pq = t; pq < kk; pq += kSpBlock) {
        const int p = pq / k, q = pq % k;
        double s = 0.0;
        for (int r = 0; r <= p; ++r) s += V[r][p] * G[r][q];
        H[p][q] = s;
    }
    __syncthreads();
    for (int pq = t; pq < kk; pq += kSpBlock) {
        const int p = pq / k, q = pq % k;
        if (p < q) {
            const double m = 0.5 * (H[p][q] + H[q][p]);
            H[p][q] = m;
            H[q][p] = m;
        }
    }
    // G <- R^{-1} (kept for M), V <- I
    for (int pq = t; pq < kk; pq += kSpBlock) {
        const int p = pq / k, q = pq % k;
        G[p][q] = V[p][q];
        V[p][q] = (p == q) ? 1.0 : 0.0;
    }
    __syncthreads();
    // parallel cyclic Jacobi (round-robin pairing over an even count ke)
    const int ke = (k + 1) & ~1;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (t == 0) {
            double o = 0.0, dd = 0.0;
            for (int p = 0; p < k; ++p)
                for (int q = 0; q < k; ++q) {
                    if (p == q) dd += H[p][p] * H[p][p];
                    else o += H[p][q] * H[p][q];
                }
            offsum = (o <= 1e-30 * (dd > 1e-300 ? dd : 1e-300)) ? -1.0 : o;
        }
        __syncthreads();
        if (offsum < 0.0) break;
        for (int round = 0; round < ke - 1; ++round) {
            // pairing of round r: position 0 fixed, the others rotate
            if (t < ke) {
                const int pos = t;
                int who;
                if (pos == 0) who = 0;
                else who = 1 + ((pos - 1 + round) % (ke - 1));
                pairs[pos] = who;
            }
            __syncthreads();
            if (t < ke / 2) {
                int p = pairs[t], q = pairs[ke - 1 - t];
                if (p > q) { const int x = p; p = q; q = x; }
                double c = 1.0, s = 0.0;
                if (q < k && fabs(H[p][q]) > 1e-300) {
                    const double tau = (H[q][q] - H[p][p]) / (2.0 * H[p][q]);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                }
                cs[t][0] = c;
                cs[t][1] = s;
            }
            __syncthreads();
            // rows: H <- J^T H for every pair (rows p and q)
            for (int e = t; e < (ke / 2) * k; e += kSpBlock) {
                const int pr = e / k, col = e % k;
                int p = pairs[pr], q = pairs[ke - 1 - pr];
                if (p > q) { const int x = p; p = q; q = x; }
                if (q < k) {
                    const double c = cs[pr][0], s = cs[pr][1];
                    const double hp = H[p][col], hq = H[q][col];
                    H[p][col] = c * hp - s * hq;
                    H[q][col] = s * hp + c * hq;
                }
            }
            __syncthreads();
            // columns: H <- H J, V <- V J
            for (int e = t; e < (ke / 2) * k; e += kSpBlock) {
                const int pr = e / k, row = e % k;
                int p = pairs[pr], q = pairs[ke - 1 - pr];
                if (p > q) { const int x = p; p = q; q = x; }
                if (q < k) {
                    const double c = cs[pr][0], s = cs[pr][1];
                    const double hp = H[row][p], hq = H[row][q];
                    H[row][p] = c * hp - s * hq;
                    H[row][q] = s * hp + c * hq;
                    const double vp = V[row][p], vq = V[row][q];
                    V[row][p] = c * vp - s * vq;
                    V[row][q] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
    }
    // order by decreasing eigenvalue (selection, one thread), then M = R^{-1} V
    if (t == 0) {
        for (int p = 0; p < k; ++p) pairs[p] = p;
        for (int a = 0; a < k; ++a) {
            int best = a;
            for (int b = a + 1; b < k; ++b)
                if (H[pairs[b]][pairs[b]] > H[pairs[best]][pairs[best]]) best = b;
            const int x = pairs[a];
            pairs[a] = pairs[best];
            pairs[best] = x;
        }
        for (int a = 0; a < k; ++a) theta[a] = H[pairs[a]][pairs[a]];
        flag[0] = bad ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int pq = t; pq < kk; pq += kSpBlock) {
        const int p = pq / k, q = pq % k;
        const int src = pairs[q];
        double s = 0.0;
        for (int r = p; r < k; ++r) s += G[p][r] * V[r][src];
        M[p * k + q] = s;
    }
}

// Y <- Y M and Z <- Z M on rows (M k x k row-major).
__global__ __launch_bounds__(kSpBlock) void k_sp_apply(double* __restrict__ Y, double* __restrict__ Z,
                                                       int64_t n, int k, const double* __restrict__ M) {
    __shared__ double Ms[kSpMaxK * kSpMaxK];
    for (int e = threadIdx.x; e < k * k; e += kSpBlock) Ms[e] = M[e];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    if (j >= n) return;
    double yr[kSpMaxK], zr[kSpMaxK];
    for (int p = 0; p < k; ++p) {
        yr[p] = Y[j * k + p];
        zr[p] = Z[j * k + p];
    }
    for (int q = 0; q < k; ++q) {
        double sy = 0.0, sz = 0.0;
        for (int p = 0; p < k; ++p) {
            sy += yr[p] * Ms[p * k + q];
            sz += zr[p] * Ms[p * k + q];
        }
        Y[j * k + q] = sy;
        Z[j * k + q] = sz;
    }
}

// Partial sums of ||Z_q - theta_q Y_q||^2 for q < c over row chunks.
__global__ __launch_bounds__(kSpBlock) void k_sp_resid(const double* __restrict__ Y,
                                                       const double* __restrict__ Z,
                                                       const double* __restrict__ theta, int64_t n,
                                                       int k, int c, double* __restrict__ part) {
    __shared__ double red[4][kSpMaxK];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    for (int q = 0; q < c; ++q) {
        double r = 0.0;
        if (j < n) {
            const double v = Z[j * k + q] - theta[q] * Y[j * k + q];
            r = v * v;
        }
        r = wsum(r);
        if (lane == 0) red[wave][q] = r;
    }
    __syncthreads();
    if (threadIdx.x < c)
        part[(int64_t)blockIdx.x * c + threadIdx.x] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// out[0] = max over q < c of the summed residual partials (squared norms),
// out[1] = the smallest Ritz value of the block, out[2] = the breakdown flag.
__global__ __launch_bounds__(kSpBlock) void k_sp_resid_max(const double* __restrict__ part, int nparts,
                                                           int c, const double* __restrict__ theta_last,
                                                           const double* __restrict__ flag,
                                                           double* __restrict__ out) {
    __shared__ double r[kSpMaxK];
    if (threadIdx.x < c) {
        double s = 0.0;
        for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * c + threadIdx.x];
        r[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int q = 0; q < c; ++q) m = r[q] > m ? r[q] : m;
        out[0] = m;
        out[1] = theta_last[0];
        out[2] = flag[0];
    }
}

// Initial block: Y[j][q] uniform in [-1, 1) from splitmix64 of (seed, j k + q).
__global__ __launch_bounds__(kSpBlock) void k_sp_init(double* __restrict__ Y, int64_t nk,
                                                      uint64_t seed) {
    const int64_t e = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    if (e >= nk) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL * (uint64_t)(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    Y[e] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

// emb[q + j c] = Y[j][q] / ||Y[j][0..c)|| (zero rows stay zero), q < c.
__global__ __launch_bounds__(kSpBlock) void k_sp_embed(const double* __restrict__ Y, int64_t n, int k,
                                                       int c, double* __restrict__ emb) {
    const int64_t j = (int64_t)blockIdx.x * kSpBlock + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int q = 0; q < c; ++q) s += Y[j * k + q] * Y[j * k + q];
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int q = 0; q < c; ++q) emb[j * c + q] = Y[j * k + q] * inv;
}

inline unsigned blocks_for(int64_t count) { return (unsigned)((count + kSpBlock - 1) / kSpBlock); }

}  // namespace

int spectral_block(int64_t n, int c) {
    const int64_t k = (int64_t)c + 8;
    return (int)(k < n ? k : n);
}

template <typename T>
respca_status spectral_embed(respca_handle h, const T* Y, int64_t ldy, int64_t d, int64_t n, int c,
                             double sigma, uint64_t seed, double* emb, SpectralStats* stats,
                             hipStream_t st, bool warm) {
    const int k = spectral_block(n, c);
    const int64_t nk = n * (int64_t)k;
    CKS(ensure(h, h->sp_w, (size_t)n * (size_t)n * sizeof(double)));
    CKS(ensure(h, h->sp_q, (size_t)n * sizeof(double)));
    CKS(ensure(h, h->sp_s, (size_t)n * sizeof(double)));
    CKS(ensure(h, h->sp_y, (size_t)nk * sizeof(double)));
    CKS(ensure(h, h->sp_z, (size_t)nk * sizeof(double)));
    CKS(ensure(h, h->sp_yp, (size_t)nk * sizeof(double)));
    CKS(ensure(h, h->sp_t, (size_t)nk * sizeof(double)));
    // block-product split: enough workgroups to fill the chip
    const int64_t rblocks = (n + 63) / 64;
    int64_t splits = (2048 + rblocks - 1) / rblocks;
    if (splits > 64) splits = 64;
    if (splits > n) splits = n;
    const int64_t jchunk = (n + splits - 1) / splits;
    splits = (n + jchunk - 1) / jchunk;
    const int64_t grows = 256;   // rows per Gram partial
    const int64_t gparts = (n + grows - 1) / grows;
    const int64_t rparts = (n + kSpBlock - 1) / kSpBlock;
    size_t part_bytes = (size_t)splits * nk * sizeof(double);
    const size_t gbytes = (size_t)gparts * 2 * k * k * sizeof(double);
    if (gbytes > part_bytes) part_bytes = gbytes;
    if ((size_t)rparts * c * sizeof(double) > part_bytes) part_bytes = (size_t)rparts * c * sizeof(double);
    CKS(ensure(h, h->sp_part, part_bytes));
    CKS(ensure(h, h->sp_small, (size_t)(k * k + k + 8) * sizeof(double)));
    CKS(ensure_spectral_status(h));
    double* W = (double*)h->sp_w.p;
    double* q = (double*)h->sp_q.p;
    double* s = (double*)h->sp_s.p;
    double* Yb = (double*)h->sp_y.p;
    double* Zb = (double*)h->sp_z.p;
    double* Yp = (double*)h->sp_yp.p;
    double* Tb = (double*)h->sp_t.p;
    double* P = (double*)h->sp_part.p;
    double* M = (double*)h->sp_small.p;
    double* theta = M + k * k;
    double* flag = theta + k;
    double* hst = h->sp_status;         // pinned host words the kernels write
    double* dst = h->sp_status_dev;

    // column norms; for a relative width (sigma < 0) the spread of the columns
    const unsigned cb = (unsigned)((n + 3) / 4);
    double width = sigma;
    if (sigma > 0.0) {
        k_sp_colsq<T><<<cb, kSpBlock, 0, st>>>(Y, ldy, d, n, q, nullptr, nullptr);
    } else {
        // column sums over splits (the n-vector s holds the deviations afterwards)
        int64_t rsplits = 64;
        if (rsplits > n) rsplits = n;
        const int64_t rchunk = (n + rsplits - 1) / rsplits;
        rsplits = (n + rchunk - 1) / rchunk;
        CKS(ensure(h, h->sp_mean, (size_t)d * (rsplits + 1) * sizeof(double)));
        double* rpart = (double*)h->sp_mean.p + d;
        double* mean = (double*)h->sp_mean.p;
        k_sp_rowsum<T><<<dim3((unsigned)((d + kSpBlock - 1) / kSpBlock), (unsigned)rsplits), kSpBlock,
                         0, st>>>(Y, ldy, d, n, rchunk, rpart);
        k_sp_mean<<<(unsigned)((d + kSpBlock - 1) / kSpBlock), kSpBlock, 0, st>>>(rpart, (int)rsplits, d,
                                                                               n, mean);
        k_sp_colsq<T><<<cb, kSpBlock, 0, st>>>(Y, ldy, d, n, q, mean, s);
        k_sp_spread<<<1, kSpBlock, 0, st>>>(s, n, dst);
        CK(hipGetLastError());
        CK(hipStreamSynchronize(st));
        const volatile double* w = hst;
        width = -sigma * std::sqrt(w[3]);
    }
    const unsigned tb = (unsigned)((n + kGramTile - 1) / kGramTile);
    // a zero width (all columns equal) makes every distance zero: W = 1 off the diagonal
    const double inv2s2 = width > 0.0 ? 1.0 / (2.0 * width * width) : 0.0;
    {
        // algorithmic work: the upper triangle of the Gram matrix, n (n + 1) d products
        ProfScope ps(h, st, RESPCA_KERNEL_AFFINITY, (double)d * n * sizeof(T) + 8.0 * (double)n * n,
                     (double)n * (double)(n + 1) * (double)d);
        k_sp_affinity<T><<<dim3(tb, tb), kSpBlock, 0, st>>>(Y, ldy, d, n, q, inv2s2, W);
    }
    k_sp_degree<<<cb, kSpBlock, 0, st>>>(W, n, s);
    // A = D^-1/2 W D^-1/2 is never formed: each block product scales the rows of Y
    // by s on the way into LDS and the rows of the result by s at the end

    auto product = [&](const double* in, double* out) {
        ProfScope ps(h, st, RESPCA_KERNEL_EIGEN, 8.0 * (double)n * n, 2.0 * (double)n * n * k);
        const dim3 g((unsigned)rblocks, (unsigned)splits);
        if (k <= 16) k_sp_mv_mfma<1><<<g, kSpBlock, 0, st>>>(W, n, in, k, jchunk, s, P);
        else if (k <= 32) k_sp_mv_mfma<2><<<g, kSpBlock, 0, st>>>(W, n, in, k, jchunk, s, P);
        else k_sp_mv_mfma<3><<<g, kSpBlock, 0, st>>>(W, n, in, k, jchunk, s, P);
        k_sp_mv_reduce<<<blocks_for(nk), kSpBlock, 0, st>>>(P, (int)splits, nk, k, s, out);
    };
    auto rayleigh_ritz = [&]() {   // on (Yb, Zb = A Yb): orthonormal Ritz vectors, theta
        for (int pass = 0; pass < 2; ++pass) {
            k_sp_gram<<<(unsigned)gparts, kSpBlock, 0, st>>>(Yb, Zb, n, k, grows, P);
            k_sp_rr<<<1, kSpBlock, 0, st>>>(P, (int)gparts, k, M, theta, flag);
            k_sp_apply<<<blocks_for(n), kSpBlock, 0, st>>>(Yb, Zb, n, k, M);
        }
    };

    if (!warm)   // else the previous call's Ritz vectors (same n and k) start the iteration
        k_sp_init<<<blocks_for(nk), kSpBlock, 0, st>>>(Yb, nk, seed ^ 0x5EC7A1C1A5731B5DULL);
    product(Yb, Zb);
    rayleigh_ritz();
    const double tol2 = 1e-20;   // squared residual norm of each wanted Ritz pair
    int it = 0;
    bool converged = false;
    double last = 0.0;
    for (it = 0; it < kSpectralMaxIters; ++it) {
        k_sp_resid<<<(unsigned)rparts, kSpBlock, 0, st>>>(Yb, Zb, theta, n, k, c, P);
        k_sp_resid_max<<<1, kSpBlock, 0, st>>>(P, (int)rparts, c, theta + (k - 1), flag, dst);
        CK(hipGetLastError());
        CK(hipStreamSynchronize(st));
        const volatile double* w = hst;
        last = w[0];
        if (w[2] != 0.0)
            return fail(h, RESPCA_ERR_INVALID,
                        "spectral p-step: the eigen block lost rank (repeated columns with sigma too small?)");
        if (last <= tol2 || k == n) {
            converged = true;
            break;
        }
        // Chebyshev filter damping [-1, b], b = the smallest Ritz value of the block
        double b = w[1];
        if (b < 0.0) b = 0.0;
        if (b > 0.999) b = 0.999;
        const double a = -1.0;
        const double e = 0.5 * (b - a), c0 = 0.5 * (b + a);
        const double x = (1.0 - c0) / e;
        int m = (int)std::floor(9.9 / std::acosh(x));   // amplification of lambda = 1 kept <~ 1e4
        if (m < 2) m = 2;
        if (m > 16) m = 16;
        // Zb holds A Yb: Y1 = (A Y0 - c0 Y0) / e; Y_{j+1} = 2 (A Y_j - c0 Y_j) / e - Y_{j-1}
        k_sp_cheb<<<blocks_for(nk), kSpBlock, 0, st>>>(Zb, Yb, nullptr, c0, 1.0 / e, 0.0, nk, Tb);
        double* prev = Yb;
        double* cur = Tb;
        double* spare = Yp;
        for (int j = 1; j < m; ++j) {
            product(cur, Zb);
            k_sp_cheb<<<blocks_for(nk), kSpBlock, 0, st>>>(Zb, cur, prev, c0, 2.0 / e, 1.0, nk, spare);
            double* x0 = prev;
            prev = cur;
            cur = spare;
            spare = x0;
        }
        if (cur != Yb) CK(hipMemcpyAsync(Yb, cur, (size_t)nk * sizeof(double), hipMemcpyDeviceToDevice, st));
        product(Yb, Zb);
        rayleigh_ritz();
    }
    k_sp_embed<<<blocks_for(n), kSpBlock, 0, st>>>(Yb, n, k, c, emb);
    if (stats) {
        stats->iters += it;
        stats->calls += 1;
        if (!converged) stats->unconverged += 1;
        stats->last_residual = std::sqrt(last);
    }
    CK(hipGetLastError());
    return RESPCA_OK;
}

template respca_status spectral_embed<float>(respca_handle, const float*, int64_t, int64_t, int64_t,
                                             int, double, uint64_t, double*, SpectralStats*,
                                             hipStream_t, bool);
template respca_status spectral_embed<double>(respca_handle, const double*, int64_t, int64_t, int64_t,
                                              int, double, uint64_t, double*, SpectralStats*,
                                              hipStream_t, bool);

// Copy of the eigenvalues of the last call (k values, decreasing).
respca_status spectral_eigenvalues(respca_handle h, int64_t n, int c, double* out, hipStream_t st) {
    const int k = spectral_block(n, c);
    CK(hipMemcpyAsync(out, (double*)h->sp_small.p + k * k, (size_t)c * sizeof(double),
                      hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    return RESPCA_OK;
}

}  // namespace respca
