// Device helpers and tile bodies shared by the single-solve kernels and the
// batched persistent kernel.  Every tile works on a slice of kRowsPerBlock
// consecutive rows of column-major d x n arrays; each wave64 load touches 64
// consecutive rows of one column, V elements per lane (16-byte vectors when d
// and the leading dimensions allow it).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace respca {

// ------------------------------------------------------------ small helpers

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum of 3 values over a 256-thread block; result valid in thread 0.  Safe to
// call repeatedly; every thread of the block must call it.
__device__ inline void block_sum3(double& a, double& b, double& c) {
    __shared__ double sh[3][kBlock / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();   // a previous call's readers are done with sh
    if (lane == 0) { sh[0][w] = a; sh[1][w] = b; sh[2][w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = sh[0][0]; b = sh[1][0]; c = sh[2][0];
        for (int i = 1; i < kBlock / 64; ++i) { a += sh[0][i]; b += sh[1][i]; c += sh[2][i]; }
    }
}

template <typename T, int V> struct Vec;
template <> struct Vec<float, 4> { using type = float4; };
template <> struct Vec<double, 2> { using type = double2; };

template <typename T, int V>
__device__ inline void vload(const T* p, T (&r)[V]) {
    if constexpr (V == 1) {
        r[0] = *p;
    } else {
        using VT = typename Vec<T, V>::type;
        VT v = *reinterpret_cast<const VT*>(p);
        if constexpr (V == 4) { r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w; }
        else { r[0] = v.x; r[1] = v.y; }
    }
}

template <typename T, int V>
__device__ inline void vload_nt(const T* p, T (&r)[V]) {
    if constexpr (V == 1) {
        r[0] = __builtin_nontemporal_load(p);
    } else {
        typedef T NV __attribute__((ext_vector_type(V)));
        const NV v = __builtin_nontemporal_load(reinterpret_cast<const NV*>(p));
#pragma unroll
        for (int e = 0; e < V; ++e) r[e] = v[e];
    }
}

template <typename T, int V>
__device__ inline void vstore_nt(T* p, const T (&r)[V]) {
    if constexpr (V == 1) {
        __builtin_nontemporal_store(r[0], p);
    } else {
        typedef T NV __attribute__((ext_vector_type(V)));
        NV v;
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = r[e];
        __builtin_nontemporal_store(v, reinterpret_cast<NV*>(p));
    }
}

template <typename T, int V>
__device__ inline void vstore(T* p, const T (&r)[V]) {
    if constexpr (V == 1) {
        *p = r[0];
    } else {
        using VT = typename Vec<T, V>::type;
        VT v;
        if constexpr (V == 4) { v.x = r[0]; v.y = r[1]; v.z = r[2]; v.w = r[3]; }
        else { v.x = r[0]; v.y = r[1]; }
        *reinterpret_cast<VT*>(p) = v;
    }
}

// Loads and stores of the streamed d x n arrays.  NT marks them nontemporal: for
// arrays far beyond the last-level cache, where nothing is reused before it is
// evicted, this raised a three-read, two-write stream from 5.6 to 6.0 TB/s.
template <bool NT, typename T, int V>
__device__ inline void sload(const T* p, T (&r)[V]) {
    if constexpr (NT) vload_nt<T, V>(p, r);
    else vload<T, V>(p, r);
}

template <bool NT, typename T, int V>
__device__ inline void sstore(T* p, const T (&r)[V]) {
    if constexpr (NT) vstore_nt<T, V>(p, r);
    else vstore<T, V>(p, r);
}

// ||y_j - y_s||^2 in double, one wave: lane partials over a fixed row order
// (U loads in flight per lane), then the wave sum.  Every seeding kernel uses
// this order, so a distance has the same value whichever kernel computes it.
// STATS: also this lane's share of ||y_j||^2 (nn) and max |y_j| (mx).
template <typename T, int V, bool STATS = false>
__device__ inline double d2_column(const T* __restrict__ yj, const T* __restrict__ ys, int64_t d,
                                   int lane, double* nn = nullptr, float* mx = nullptr) {
    double acc = 0.0;
    constexpr int U = 4;
    auto stats = [&](T a) {
        if constexpr (STATS) {
            *nn += (double)a * (double)a;
            *mx = fmaxf(*mx, fabsf((float)a));
        }
    };
    int64_t i = (int64_t)lane * V;
    for (; i + (int64_t)64 * V * (U - 1) < d; i += (int64_t)64 * V * U) {
        T a[U][V], b[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vload<T, V>(yj + i + (int64_t)64 * V * u, a[u]);
            vload<T, V>(ys + i + (int64_t)64 * V * u, b[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double t = (double)a[u][v] - (double)b[u][v];
                acc += t * t;
                stats(a[u][v]);
            }
    }
    for (; i < d; i += 64 * V) {
        T a[V], b[V];
        vload<T, V>(yj + i, a);
        vload<T, V>(ys + i, b);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double t = (double)a[v] - (double)b[v];
            acc += t * t;
            stats(a[v]);
        }
    }
    return wave_sum(acc);
}

// d2_column<float, 4> of NC columns against the same seed column, computed
// together: every 512-row pass issues the seed's loads once and all the columns'
// loads before any arithmetic.  Each lane visits its rows in the same order as
// d2_column, so every result is bitwise that of d2_column.  d % 4 == 0.
template <int NC>
__device__ inline void d2_columns(const float* const (&yj)[NC], const float* __restrict__ ys,
                                  int64_t d, int lane, double (&out)[NC]) {
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    constexpr int U = 2;
    int64_t i = (int64_t)lane * 4;
    for (; i + 256 * (U - 1) < d; i += 256 * U) {
        float b[U][4], a[NC][U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) vload<float, 4>(ys + i + 256 * u, b[u]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int u = 0; u < U; ++u) vload<float, 4>(yj[c] + i + 256 * u, a[c][u]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double t = (double)a[c][u][v] - (double)b[u][v];
                    acc[c] += t * t;
                }
    }
    for (; i < d; i += 256) {
        float b[4], a[NC][4];
        vload<float, 4>(ys + i, b);
#pragma unroll
        for (int c = 0; c < NC; ++c) vload<float, 4>(yj[c] + i, a[c]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double t = (double)a[c][v] - (double)b[v];
                acc[c] += t * t;
            }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = wave_sum(acc[c]);
}

// The column indices of one group segment (at most kMaxSegCols), copied from the
// sort permutation into LDS once per tile so that the column loop does not wait
// on a global load before each batch of columns.  Every thread must call it.
constexpr int kMaxSegCols = 64;
__device__ inline const int32_t* stage_segment_cols(const int32_t* __restrict__ perm, int begin,
                                                    int len) {
    __shared__ int32_t cols[kMaxSegCols];
    __syncthreads();   // the previous tile's readers are done
    for (int q = threadIdx.x; q < len; q += kBlock) cols[q] = perm[begin + q];
    __syncthreads();
    return cols;
}

// LDS buffer for the column groups' partial sums below, shared by every
// instantiation (one allocation per kernel).
constexpr int kGroupRedDoubles = 1024;
__device__ inline double* group_red_lds() {
    __shared__ double red[kGroupRedDoubles];
    return red;
}

// ------------------------------------------------------------- tile bodies

// The fused ALM sweep over columns [j0, j1) of rows [r0, r0 + ROWS).  The block's
// threads form CG column groups of kBlock / CG threads; group g takes columns
// j0 + g, j0 + g + CG, ... (CG > 1 keeps all lanes busy when d is small).
// Per entry (i, j) with group p = labels[j]:
//   D  = X - S + Theta/rho                     (matrix the L-step pulls toward)
//   L  = alpha D + beta C[:, p]                (Sec. 4.1 closed form, C = group mean of D)
//   B  = X - L + Theta/rho;  S' = sign(B) max(|B| - 1/rho, 0)      (Sec. 4.3)
//   Theta' = Theta + rho (X - L - S')                              (Sec. 4.4)
// and adds this thread's squared norms of X - L - S', L - L_prev, S' - S to a0..a2.
template <typename T, int V, int ROWS = kRowsPerBlock, int CG = 1>
__device__ inline void sweep_tile(const T* __restrict__ X, int64_t ldx, T* __restrict__ L,
                                  int64_t ldl, T* __restrict__ S, int64_t lds, T* __restrict__ Th,
                                  int64_t ldt, const T* __restrict__ C,
                                  const int32_t* __restrict__ labels, int64_t d, int64_t j0,
                                  int64_t j1, int64_t r0, T alpha, T beta, T rho, T inv_rho,
                                  double& a0, double& a1, double& a2) {
    constexpr int TPC = kBlock / CG;   // threads per column group
    constexpr int NS = ROWS / (TPC * V);
    static_assert(NS >= 1 && NS * TPC * V == ROWS, "row block must tile the column group");
    constexpr int U = 2;   // columns in flight per thread (columns are independent)
    const int cg = (int)threadIdx.x / TPC, tl = (int)threadIdx.x % TPC;
    for (int64_t jb = j0 + cg; jb < j1; jb += (int64_t)U * CG) {
        int64_t pp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pp[u] = (jb + u * CG < j1) ? labels[jb + u * CG] : 0;
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const int64_t i = r0 + (int64_t)(a * TPC + tl) * V;
            if (i >= d) continue;
            T xs[U][V], ss[U][V], ts[U][V], lps[U][V], ms[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (jb + u * CG >= j1) continue;
                const int64_t j = jb + u * CG;
                vload<T, V>(X + j * ldx + i, xs[u]);
                vload<T, V>(S + j * lds + i, ss[u]);
                vload<T, V>(Th + j * ldt + i, ts[u]);
                vload<T, V>(L + j * ldl + i, lps[u]);
                vload<T, V>(C + pp[u] * d + i, ms[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
            if (jb + u * CG >= j1) continue;
            const int64_t j = jb + u * CG;
            const T (&x)[V] = xs[u];
            const T (&s)[V] = ss[u];
            const T (&t)[V] = ts[u];
            const T (&lp)[V] = lps[u];
            const T (&m)[V] = ms[u];
            T ln[V], sn[V], tn[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const T dv = x[v] - s[v] + t[v] * inv_rho;
                ln[v] = alpha * dv + beta * m[v];
                const T b = x[v] - ln[v] + t[v] * inv_rho;
                const T mag = fabs(b) - inv_rho;
                sn[v] = mag > T(0) ? copysign(mag, b) : T(0);
                const T r = x[v] - ln[v] - sn[v];
                tn[v] = t[v] + rho * r;
                const double dl = (double)ln[v] - (double)lp[v];
                const double ds = (double)sn[v] - (double)s[v];
                a0 += (double)r * (double)r;
                a1 += dl * dl;
                a2 += ds * ds;
            }
            vstore<T, V>(L + j * ldl + i, ln);
            vstore<T, V>(S + j * lds + i, sn);
            vstore<T, V>(Th + j * ldt + i, tn);
            }
        }
    }
}

// The l1 proximal step and the multiplier it leaves: soft(b, tau) =
// sign(b) max(|b| - tau, 0), and clip(t) = t clamped to [-1, 1] (a NaN stays NaN).
template <typename T>
__device__ inline T soft_threshold(T b, T tau) {
    const T mag = fabs(b) - tau;
    return mag > T(0) ? copysign(mag, b) : T(0);
}

template <typename T>
__device__ inline T clip_unit(T t) {
    return t > T(1) ? T(1) : (t < T(-1) ? T(-1) : t);
}

// The fused sweep over one group segment: the `len` columns perm[begin..) (all in
// group p) over rows [r0, r0 + ROWS), CG column groups of kBlock / CG threads
// (group g takes the segment's columns g, g + CG, ...), U columns in flight.  Per
// entry it does what sweep_tile does and also sums D' = X - S' + Theta' * inv_rho_next
// over the segment's columns -- the group sums of the next L-step when the p-step
// keeps every label -- in the order and arithmetic of group_partial_tile (column
// groups added in group order), written to out[i] (this segment's d-vector).
// L21: the column-wise (l2,1) S-step, S_j = fac[j] B_j with the per-column factor
// max(0, 1 - 1/(rho ||B_j||)) computed beforehand over the whole column.
// COMPACT (l1 only): the state is B = X - L + Theta_old / rho, kept in S (Th is
// not used).  The l1 S-step and the multiplier update are functions of B alone:
// S = soft(B, 1/rho) and Theta_old + rho (X - L - S) = rho (B - S) = clip(rho B), so
// S and Theta of the previous iteration are recovered from its B with its
// penalty rho_prev, and the sweep reads X, B, L and writes L, B (five d x n
// streams instead of seven).
template <typename T, int V, int ROWS, int CG, int U, bool L21 = false, bool COMPACT = false,
          bool NT = false>
__device__ inline void seg_sweep_tile(const T* __restrict__ X, int64_t ldx, T* __restrict__ L,
                                      int64_t ldl, T* __restrict__ S, int64_t lds,
                                      T* __restrict__ Th, int64_t ldt, const T* __restrict__ C,
                                      int64_t p, int64_t d, const int32_t* __restrict__ perm,
                                      int begin, int len, int64_t r0, T alpha, T beta, T rho,
                                      T inv_rho, T inv_rho_next, double& a0, double& a1, double& a2,
                                      double* __restrict__ out,
                                      const double* __restrict__ fac = nullptr,
                                      T rho_prev = T(0), T inv_rho_prev = T(0)) {
    static_assert(!(COMPACT && L21), "the compact state holds the l1 form only");
    constexpr int TPC = kBlock / CG;
    constexpr int NS = ROWS / (TPC * V);
    static_assert(NS >= 1 && NS * TPC * V == ROWS, "row block must tile the column group");
    const int cg = (int)threadIdx.x / TPC, tl = (int)threadIdx.x % TPC;
    const int32_t* cols = stage_segment_cols(perm, begin, len);
    double acc[NS][V];
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[a][v] = 0.0;
    // One step: U columns of the segment (FULL: all inside it, so no load sits
    // behind a branch and the waits before each column's stores stay exact).
    auto step = [&](int q0, auto full) {
        constexpr bool FULL = decltype(full)::value;
        int64_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jj[u] = (FULL || q0 + u * CG < len) ? cols[q0 + u * CG] : -1;
        T fu[U];
        if constexpr (L21) {
#pragma unroll
            for (int u = 0; u < U; ++u) fu[u] = (FULL || jj[u] >= 0) ? (T)fac[jj[u]] : T(0);
        }
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const int64_t i = r0 + (int64_t)(a * TPC + tl) * V;
            if (i >= d) continue;
            T xs[U][V], ss[U][V], ts[U][V], lps[U][V], m[V];
            vload<T, V>(C + p * d + i, m);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!FULL && jj[u] < 0) continue;
                sload<NT, T, V>(X + jj[u] * ldx + i, xs[u]);
                sload<NT, T, V>(S + jj[u] * lds + i, ss[u]);
                if constexpr (!COMPACT) sload<NT, T, V>(Th + jj[u] * ldt + i, ts[u]);
                sload<NT, T, V>(L + jj[u] * ldl + i, lps[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!FULL && jj[u] < 0) continue;
                const int64_t j = jj[u];
                T ln[V], sn[V], tn[V], bn[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T x = xs[u][v];
                    T sv, t;
                    if constexpr (COMPACT) {
                        sv = soft_threshold(ss[u][v], inv_rho_prev);
                        t = clip_unit(rho_prev * ss[u][v]);
                    } else {
                        sv = ss[u][v];
                        t = ts[u][v];
                    }
                    const T dv = x - sv + t * inv_rho;
                    ln[v] = alpha * dv + beta * m[v];
                    const T b = x - ln[v] + t * inv_rho;
                    if constexpr (L21) {
                        sn[v] = fu[u] * b;
                    } else {
                        const T mag = fabs(b) - inv_rho;
                        sn[v] = mag > T(0) ? copysign(mag, b) : T(0);
                    }
                    const T rr = x - ln[v] - sn[v];
                    tn[v] = COMPACT ? clip_unit(rho * b) : t + rho * rr;
                    bn[v] = b;
                    const double dl = (double)ln[v] - (double)lps[u][v];
                    const double ds = (double)sn[v] - (double)sv;
                    a0 += (double)rr * (double)rr;
                    a1 += dl * dl;
                    a2 += ds * ds;
                    acc[a][v] += (double)(x - sn[v] + tn[v] * inv_rho_next);
                }
                sstore<NT, T, V>(L + j * ldl + i, ln);
                if constexpr (COMPACT) {
                    sstore<NT, T, V>(S + j * lds + i, bn);
                } else {
                    sstore<NT, T, V>(S + j * lds + i, sn);
                    sstore<NT, T, V>(Th + j * ldt + i, tn);
                }
            }
        }
    };
    int q0 = cg;
    for (; q0 + (U - 1) * CG < len; q0 += U * CG) step(q0, std::true_type{});
    if (q0 < len) step(q0, std::false_type{});   // the segment's last, partial step
    if constexpr (CG == 1) {
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const int64_t i = r0 + (int64_t)(a * TPC + tl) * V;
            if (i < d)
#pragma unroll
                for (int v = 0; v < V; ++v) out[i + v] = acc[a][v];
        }
    } else {
        static_assert(CG * ROWS <= kGroupRedDoubles, "partial-sum buffer too small");
        double* red = group_red_lds();
#pragma unroll
        for (int a = 0; a < NS; ++a)
#pragma unroll
            for (int v = 0; v < V; ++v) red[cg * ROWS + (a * TPC + tl) * V + v] = acc[a][v];
        __syncthreads();
        for (int e = threadIdx.x; e < ROWS; e += kBlock) {
            if (r0 + e < d) {
                double t = red[e];
#pragma unroll
                for (int g = 1; g < CG; ++g) t += red[g * ROWS + e];
                out[r0 + e] = t;
            }
        }
        __syncthreads();   // red is reused by the next call
    }
}

// Sum over the `len` columns perm[begin..begin+len) (one group segment) of
// Y = X - S + Theta*inv_rho (WITH_D) or Y = A, rows [r0, r0 + ROWS), in double,
// written to out[i] (out points at this segment's d-vector).  With CG column
// groups, group g sums the segment's columns g, g + CG, ... and the CG partial
// sums are added in group order at the end; the order of every sum is fixed.
// COMPACT (with D): S holds the compact state B of the previous sweep (penalty
// rho_prev), from which D = X - soft(B, 1/rho_prev) + clip(rho_prev B) * inv_rho.
template <typename T, int V, bool WITH_D, int ROWS = kRowsPerBlock, int CG = 1, bool COMPACT = false,
          bool NT = false>
__device__ inline void group_partial_tile(const T* __restrict__ A, int64_t lda,
                                          const T* __restrict__ S, int64_t lds,
                                          const T* __restrict__ Th, int64_t ldt, T inv_rho,
                                          int64_t d, const int32_t* __restrict__ perm, int begin,
                                          int len, int64_t r0, double* __restrict__ out,
                                          T rho_prev = T(0), T inv_rho_prev = T(0)) {
    constexpr int TPC = kBlock / CG;
    constexpr int NS = ROWS / (TPC * V);
    static_assert(NS >= 1 && NS * TPC * V == ROWS, "row block must tile the column group");
    // columns in flight per thread (each a load of A, and of S and Theta with D);
    // the summation order is unchanged
    constexpr int U = WITH_D ? 4 : 8;
    const int cg = (int)threadIdx.x / TPC, tl = (int)threadIdx.x % TPC;
    double acc[NS][V];
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[a][v] = 0.0;
    auto value = [&](int64_t j, int64_t i, T (&x)[V]) {
        sload<NT, T, V>(A + j * lda + i, x);
        if constexpr (WITH_D && COMPACT) {
            T bv[V];
            sload<NT, T, V>(S + j * lds + i, bv);
#pragma unroll
            for (int v = 0; v < V; ++v)
                x[v] = x[v] - soft_threshold(bv[v], inv_rho_prev) + clip_unit(rho_prev * bv[v]) * inv_rho;
        } else if constexpr (WITH_D) {
            T sv[V], tv[V];
            sload<NT, T, V>(S + j * lds + i, sv);
            sload<NT, T, V>(Th + j * ldt + i, tv);
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = x[v] - sv[v] + tv[v] * inv_rho;
        }
    };
    const int32_t* cols = stage_segment_cols(perm, begin, len);
    // U columns per step; past the segment's end the last column is loaded again
    // (unconditional loads) and its values are not added
    for (int q = cg; q < len; q += U * CG) {
        int64_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jj[u] = cols[q + u * CG < len ? q + u * CG : len - 1];
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const int64_t i = r0 + (int64_t)(a * TPC + tl) * V;
            if (i < d) {
                T x[U][V];
#pragma unroll
                for (int u = 0; u < U; ++u) value(jj[u], i, x[u]);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (q + u * CG < len)
#pragma unroll
                        for (int v = 0; v < V; ++v) acc[a][v] += (double)x[u][v];
            }
        }
    }
    if constexpr (CG == 1) {
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const int64_t i = r0 + (int64_t)(a * TPC + tl) * V;
            if (i < d)
#pragma unroll
                for (int v = 0; v < V; ++v) out[i + v] = acc[a][v];
        }
    } else {
        static_assert(CG * ROWS <= kGroupRedDoubles, "partial-sum buffer too small");
        double* red = group_red_lds();
#pragma unroll
        for (int a = 0; a < NS; ++a)
#pragma unroll
            for (int v = 0; v < V; ++v) red[cg * ROWS + (a * TPC + tl) * V + v] = acc[a][v];
        __syncthreads();
        for (int e = threadIdx.x; e < ROWS; e += kBlock) {
            if (r0 + e < d) {
                double t = red[e];
#pragma unroll
                for (int g = 1; g < CG; ++g) t += red[g * ROWS + e];
                out[r0 + e] = t;
            }
        }
        __syncthreads();   // red is reused by the next call
    }
}

}  // namespace respca
