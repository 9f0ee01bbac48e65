// The MFMA distance tile shared by the single-solve and batched kernels:
// partial products C^T Y for 128 columns x 128 groups over one slice of rows,
// staged through LDS 32 rows at a time (FP32 v_mfma_f32_16x16x4f32, or split
// bf16 hi/lo on v_mfma_f32_16x16x32_bf16).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace respca {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxCand = 8;  // candidate groups kept per near-tied column

constexpr int kJT = 128;     // columns per workgroup
constexpr int kKC = 128;     // groups per workgroup (8 blocks of 16)
constexpr int kRT = 32;      // rows per LDS stage
constexpr int kStride = 36;  // padded LDS stride (floats) of one staged column: conflict-free
constexpr int kStrideH = 40; // padded LDS stride (bf16) of one staged column (80 bytes)


// A 32-row stage of 128 consecutive columns of a column-major matrix, held in
// registers between its global load and its LDS store (zero outside the
// matrix), so that the next stage's loads are in flight during the MFMAs.
template <bool VEC>
struct StageRegs {
    float4 v4[VEC ? 4 : 1];
    float v1[VEC ? 1 : 16];
    const float* ptr[VEC ? 4 : 1];   // VEC: this thread's four columns at row 0 of the tile's rows

    // VEC: fix this thread's four column pointers once per tile (they only move by
    // rows from stage to stage).  Columns past the matrix are clamped to its last
    // column: their products only reach outputs of those columns, which nobody
    // reads, and every load stays unconditional (no branch splits the count of
    // loads in flight).
    __device__ inline void init(const float* __restrict__ src, int64_t ld, int64_t col0,
                                int64_t ncols) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            int64_t gj = col0 + p * 32 + (tid >> 3);
            if (gj >= ncols) gj = ncols - 1;
            ptr[p] = src + (tid & 7) * 4 + gj * ld;
        }
    }

    // VEC: rows [r, r + 32) of the four columns fixed by init (zero past rend;
    // rend and the row offsets are multiples of 4).  A full stage loads without
    // conditions; the last partial stage reads row 0 in place of the rows past
    // rend and zeroes them.
    // VEC: a stage known to lie inside the rows (r + 32 <= rend).
    __device__ inline void load_rows_full(int64_t r) {
#pragma unroll
        for (int p = 0; p < 4; ++p) v4[p] = *reinterpret_cast<const float4*>(ptr[p] + r);
    }

    __device__ inline void load_rows(int64_t r, int64_t rend) {
        if (r + kRT <= rend) {
            load_rows_full(r);
        } else {
            const int64_t rr = (threadIdx.x & 7) * 4;
            const bool in = r + rr < rend;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const float4 t = *reinterpret_cast<const float4*>(in ? ptr[p] + r : ptr[p] - rr);
                v4[p] = in ? t : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    }

    // Scalar layout: rows [r, r + 32) of columns [col0, col0 + 128), zero outside the
    // matrix (the VEC layout loads through init / load_rows).
    __device__ inline void load(const float* __restrict__ src, int64_t ld, int64_t col0,
                                int64_t ncols, int64_t r, int64_t rend) {
        static_assert(!VEC, "the VEC layout loads through init / load_rows");
        const int tid = threadIdx.x;
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const int e = tid + 256 * p, col = e >> 5, rr = e & 31;
            const int64_t gj = col0 + col, gi = r + rr;
            v1[p] = (gj < ncols && gi < rend) ? src[gj * ld + gi] : 0.f;
        }
    }

    // This thread's share of the sum of squares of each staged column, added to
    // acc[] (VEC: acc[p] for column p*32 + tid/8, 4 rows per lane; scalar: acc[p]
    // for column tid/32 + 8p, one row per lane); col_sumsq_reduce completes the
    // sums across the lanes that share a column once all stages are in.
    __device__ inline void col_sumsq(float* acc) const {
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
                acc[p] += v4[p].x * v4[p].x + v4[p].y * v4[p].y + v4[p].z * v4[p].z + v4[p].w * v4[p].w;
        } else {
#pragma unroll
            for (int p = 0; p < 16; ++p) acc[p] += v1[p] * v1[p];
        }
    }

    // Sums the per-lane shares: VEC over the 8 lanes of a column (valid in lanes
    // with tid % 8 == 0), scalar over its 32 lanes (valid where tid % 32 == 0).
    static __device__ inline void col_sumsq_reduce(float* acc) {
        constexpr int kLanes = VEC ? 8 : 32;
#pragma unroll
        for (int p = 0; p < (VEC ? 4 : 16); ++p)
#pragma unroll
            for (int o = 1; o < kLanes; o <<= 1) acc[p] += __shfl_xor(acc[p], o);
    }

    // Store as bf16 high and low parts (x = hi + lo + O(2^-16 x)), stride kStrideH.
    __device__ inline void store_split(__bf16* __restrict__ hi, __bf16* __restrict__ lo) const {
        const int tid = threadIdx.x;
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int col = p * 32 + (tid >> 3);
                const int rr = (tid & 7) * 4;
                const float x[4] = {v4[p].x, v4[p].y, v4[p].z, v4[p].w};
                bf16x4 h, l;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    h[e] = (__bf16)x[e];
                    l[e] = (__bf16)(x[e] - (float)h[e]);
                }
                // one 8-byte LDS store per part (rr * 2 bytes is 8-byte aligned)
                *reinterpret_cast<bf16x4*>(hi + col * kStrideH + rr) = h;
                *reinterpret_cast<bf16x4*>(lo + col * kStrideH + rr) = l;
            }
        } else {
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const int e = tid + 256 * p, col = e >> 5, rr = e & 31;
                const __bf16 h = (__bf16)v1[p];
                hi[col * kStrideH + rr] = h;
                lo[col * kStrideH + rr] = (__bf16)(v1[p] - (float)h);
            }
        }
    }

    __device__ inline void store(float* __restrict__ dst) const {
        const int tid = threadIdx.x;
        if constexpr (VEC) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int col = p * 32 + (tid >> 3);
                const int rr = (tid & 7) * 4;
                *reinterpret_cast<float4*>(dst + col * kStride + rr) = v4[p];
            }
        } else {
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const int e = tid + 256 * p, col = e >> 5, rr = e & 31;
                dst[col * kStride + rr] = v1[p];
            }
        }
    }
};

// Centroids already split into bf16 parts: element (k, g) of the [kpad][ldq]
// array holds rows 4g..4g+3 of group k as {hi[4], lo[4]} (16 bytes), zero past
// the last row, so a stage is a plain copy into the LDS hi/lo tiles.
// NT threads share the stage of the first GROUPS group columns (rounded up to
// whole passes of NT / 8 columns): thread t takes row group t % 8 of group
// columns t / 8 + (NT / 8) p.
template <int NT = 256, int GROUPS = kKC>
struct SplitStage {
    static constexpr int P = (GROUPS * 8 + NT - 1) / NT;
    static_assert(P >= 1 && P * (NT / 8) <= kKC, "at most 128 groups per stage");
    uint4 v[P];
    const uint4* ptr[P];

    // group columns past kpad are clamped to the last one (no MFMA reads them)
    __device__ inline void init(const uint4* __restrict__ Csp, int64_t ldq, int k0, int kpad) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            int gk = k0 + p * (NT / 8) + (tid >> 3);
            if (gk >= kpad) gk = kpad - 1;
            ptr[p] = Csp + (tid & 7) + (int64_t)gk * ldq;
        }
    }
    // rows [r, r + 32) (r a multiple of 32; the padded rows read as zero)
    __device__ inline void load_rows(int64_t r) {
#pragma unroll
        for (int p = 0; p < P; ++p) v[p] = ptr[p][r >> 2];
    }
    // PERM: row group rg (rows 4rg..4rg+3) goes to position 8 (rg % 4) + 4 (rg / 4),
    // so that the 8 values at 8g..8g+7 are rows 4g..4g+3 and 16+4g..16+4g+3
    // (the row order of the direct tile's K slots).
    template <bool PERM = false>
    __device__ inline void store(__bf16* __restrict__ hi, __bf16* __restrict__ lo) const {
        const int tid = threadIdx.x;
        const int rg = tid & 7;
        const int rr = PERM ? 8 * (rg & 3) + 4 * (rg >> 2) : 4 * rg;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int col = p * (NT / 8) + (tid >> 3);
            *reinterpret_cast<uint2*>(hi + col * kStrideH + rr) = make_uint2(v[p].x, v[p].y);
            *reinterpret_cast<uint2*>(lo + col * kStrideH + rr) = make_uint2(v[p].z, v[p].w);
        }
    }
};

// One distance tile: columns [j0, j0 + 128) x groups [k0, k0 + 128) over the
// rows of slice s; writes part[s][j][k] (and, with YN and write_ynorm,
// the slice's column sums of squares).  256 threads.  DB: two LDS stage
// buffers, so a stage's MFMAs and the staging of the next one share one barrier
// and can overlap (twice the LDS).  CS (bf16 only): the centroids come pre-split
// from Csp (SplitStage layout, ldq row groups per group) instead of C.
template <bool VEC, bool BF16, bool DB = false, bool CS = false, bool YN = BF16>
__device__ inline void dist_tile(const float* __restrict__ C, int64_t d, int c, int kpad,
                                 const float* __restrict__ Y, int64_t ldy, int64_t n, int slice_rows,
                                 float* __restrict__ part, float* __restrict__ ynorm_part,
                                 int64_t j0, int s, int k0, bool write_ynorm,
                                 const uint4* __restrict__ Csp = nullptr, int64_t ldq = 0) {
    static_assert(!CS || BF16, "pre-split centroids are bf16 parts");
    // fp32 mode: Ys, Cs as floats; bf16 mode: hi/lo halves of both operands.
    constexpr size_t kF32Bytes = 2 * kJT * kStride * sizeof(float);
    constexpr size_t kBf16Bytes = 2 * (kJT + kKC) * kStrideH * sizeof(__bf16);
    constexpr size_t kStage = kF32Bytes > kBf16Bytes ? kF32Bytes : kBf16Bytes;
    __shared__ __attribute__((aligned(16))) char smem[(DB ? 2 : 1) * kStage];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    __syncthreads();   // the LDS tiles may still be read by a previous tile of this workgroup
    const int q = lane & 15, g = lane >> 4;
    const int64_t r0 = (int64_t)s * slice_rows;
    const int64_t r1 = r0 + slice_rows < d ? r0 + slice_rows : d;
    const int nkb = (kpad - k0 < kKC ? kpad - k0 : kKC) / 16;
    constexpr int NCOL = VEC ? 4 : 16;
    float ycol[NCOL];
#pragma unroll
    for (int p = 0; p < NCOL; ++p) ycol[p] = 0.f;

    floatx4 acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    // Two register sets (PF2: VEC with two LDS buffers) so that a stage's loads can
    // be issued two stages ahead; otherwise only set 0 is used.
    constexpr bool PF2 = DB && VEC;
    StageRegs<VEC> ry[PF2 ? 2 : 1];
    StageRegs<VEC> rc[PF2 ? 2 : 1];   // unused with CS
    SplitStage<> rs[PF2 ? 2 : 1];
    if constexpr (VEC) ry[0].init(Y, ldy, j0, n);
    if constexpr (CS) rs[0].init(Csp, ldq, k0, kpad);
    else if constexpr (VEC) rc[0].init(C, d, k0, c);
    if constexpr (PF2) {
        ry[1] = ry[0];
        rc[1] = rc[0];
        rs[1] = rs[0];
    }
    using Set0 = std::integral_constant<int, 0>;
    using Set1 = std::integral_constant<int, PF2 ? 1 : 0>;
    auto load_stage = [&](auto set, int64_t r) {
        constexpr int S = decltype(set)::value;
        if constexpr (VEC) ry[S].load_rows(r, r1);
        else ry[S].load(Y, ldy, j0, n, r, r1);
        if constexpr (CS) rs[S].load_rows(r);
        else if constexpr (VEC) rc[S].load_rows(r, r1);
        else rc[S].load(C, d, k0, c, r, r1);
    };
    // VEC, a stage inside the rows: loads without any branch
    auto load_full = [&](auto set, int64_t r) {
        constexpr int S = decltype(set)::value;
        if constexpr (VEC) {
            ry[S].load_rows_full(r);
            if constexpr (CS) rs[S].load_rows(r);
            else rc[S].load_rows_full(r);
        }
    };
    // registers -> LDS buffer b (bf16: split into hi/lo, and the columns' sums of squares)
    auto store_stage = [&](auto set, int b) {
        constexpr int S = decltype(set)::value;
        char* base = smem + (DB ? b * kStage : 0);
        if constexpr (BF16) {
            __bf16* Yh = reinterpret_cast<__bf16*>(base);
            __bf16* Yl = Yh + kJT * kStrideH;
            __bf16* Ch = Yl + kJT * kStrideH;
            __bf16* Cl = Ch + kKC * kStrideH;
            ry[S].col_sumsq(ycol);
            ry[S].store_split(Yh, Yl);
            if constexpr (CS) rs[S].store(Ch, Cl);
            else rc[S].store_split(Ch, Cl);
        } else {
            float* Ys = reinterpret_cast<float*>(base);
            if constexpr (YN) ry[S].col_sumsq(ycol);
            ry[S].store(Ys);
            rc[S].store(Ys + kJT * kStride);
        }
    };
    // the MFMAs of the stage held in LDS buffer b
    auto mfma_stage = [&](int b) {
        const char* base = smem + (DB ? b * kStage : 0);
        if constexpr (BF16) {
            const __bf16* Yh = reinterpret_cast<const __bf16*>(base);
            const __bf16* Yl = Yh + kJT * kStrideH;
            const __bf16* Ch = Yl + kJT * kStrideH;
            const __bf16* Cl = Ch + kKC * kStrideH;
            // one 16x16x32 instruction covers the stage: lane group g holds rows 8g..8g+7
            bf16x8 ahi[2], alo[2];
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                const int col = wave * 32 + jb * 16 + q;
                ahi[jb] = *reinterpret_cast<const bf16x8*>(Yh + col * kStrideH + g * 8);
                alo[jb] = *reinterpret_cast<const bf16x8*>(Yl + col * kStrideH + g * 8);
            }
#pragma unroll
            for (int kb = 0; kb < 8; ++kb) {
                if (kb < nkb) {
                    const int row = kb * 16 + q;
                    const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(Ch + row * kStrideH + g * 8);
                    const bf16x8 blo = *reinterpret_cast<const bf16x8*>(Cl + row * kStrideH + g * 8);
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb) {
                        acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[jb], bhi, acc[jb][kb], 0, 0, 0);
                        acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[jb], blo, acc[jb][kb], 0, 0, 0);
                        acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[jb], bhi, acc[jb][kb], 0, 0, 0);
                    }
                }
            }
        } else {
            const float* Ys = reinterpret_cast<const float*>(base);
            const float* Cs = Ys + kJT * kStride;
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
                    const float b8[8] = {u.x, u.y, u.z, u.w, w.x, w.y, w.z, w.w};
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                        for (int m = 0; m < 8; ++m)
                            acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[jb][m], b8[m], acc[jb][kb], 0, 0, 0);
                }
            }
        }
    };
    if constexpr (PF2) {
        // Buffer 0 holds stage r and set 1 holds (or is loading) stage r + 32 at the
        // top of each pass.  A half-step loads stage r + 64 into the free set, runs
        // the MFMAs of the buffered stage, then stores the older set into the other
        // buffer; its loads had a whole half-step to arrive.
        if (r0 < r1) {
            load_stage(Set0{}, r0);
            store_stage(Set0{}, 0);
            if (r0 + kRT < r1) load_stage(Set1{}, r0 + kRT);
            __syncthreads();
        }
        int64_t r = r0;
        // steady state (both loaded stages inside the rows): every load
        // unconditional, so the waits before each store leave the newest set's loads
        // in flight
        for (; r + 4 * kRT <= r1; r += 2 * kRT) {
            load_full(Set0{}, r + 2 * kRT);
            mfma_stage(0);
            store_stage(Set1{}, 1);
            __syncthreads();
            load_full(Set1{}, r + 3 * kRT);
            mfma_stage(1);
            store_stage(Set0{}, 0);
            __syncthreads();
        }
        // the last one to three stages
        for (; r < r1; r += 2 * kRT) {
            if (r + 2 * kRT < r1) load_stage(Set0{}, r + 2 * kRT);
            mfma_stage(0);
            if (r + kRT < r1) store_stage(Set1{}, 1);
            __syncthreads();
            if (r + kRT >= r1) break;
            if (r + 3 * kRT < r1) load_stage(Set1{}, r + 3 * kRT);
            mfma_stage(1);
            if (r + 2 * kRT < r1) store_stage(Set0{}, 0);
            __syncthreads();
        }
    } else if constexpr (DB) {
        if (r0 < r1) {
            load_stage(Set0{}, r0);
            store_stage(Set0{}, 0);
            __syncthreads();
        }
        int b = 0;
        for (int64_t r = r0; r < r1; r += kRT, b ^= 1) {
            const bool more = r + kRT < r1;
            if (more) load_stage(Set0{}, r + kRT);   // global loads in flight during the MFMAs
            mfma_stage(b);
            if (more) store_stage(Set0{}, b ^ 1);    // the other buffer was released by the last barrier
            __syncthreads();
        }
    } else {
        if (r0 < r1) load_stage(Set0{}, r0);
        for (int64_t r = r0; r < r1; r += kRT) {
            store_stage(Set0{}, 0);
            __syncthreads();
            if (r + kRT < r1) load_stage(Set0{}, r + kRT);  // next stage's loads overlap this stage's MFMAs
            mfma_stage(0);
            __syncthreads();
        }
    }
    if constexpr (YN) {
        if (write_ynorm) {
            StageRegs<VEC>::col_sumsq_reduce(ycol);
#pragma unroll
            for (int p = 0; p < NCOL; ++p) {
                const int col = VEC ? p * 32 + (tid >> 3) : (tid >> 5) + 8 * p;
                const bool owner = VEC ? (tid & 7) == 0 : (tid & 31) == 0;
                const int64_t j = j0 + col;
                if (owner && j < n) ynorm_part[(int64_t)s * n + j] = ycol[p];
            }
        }
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


// bf16 distance tile with the column operand read straight into registers
// (VEC layout, pre-split centroids): the products of dist_tile<true, true, true,
// true> for 32 WAVES columns, each wave loading its own 32 columns in MFMA operand order and
// splits them in registers, so only the centroids pass through LDS.  The K slots
// of lane group g are rows 4g..4g+3 and 16+4g..16+4g+3 of the stage (two 16-byte
// loads per column, 64 contiguous bytes per four lanes), and the centroid tiles
// are stored in LDS in that row order.  NKB group blocks of 16 (fixed at compile
// time; blocks past the tile's groups compute on clamped copies and are not
// written): all centroid operands of a stage are read from LDS first, then the
// MFMAs run product by product over every (block, column half), so that 2 NKB
// independent accumulators separate two updates of the same one.  AHEAD: stages
// of column values in flight beyond the one being multiplied (1 or 2; with 2 a
// step issues the next stage's centroid loads before the values two stages
// ahead, so that the centroid wait at its end leaves those in flight).
template <int NKB, int WAVES, int AHEAD>
__device__ inline void dist_tile_ydirect(int64_t d, int kpad, const float* __restrict__ Y,
                                         int64_t ldy, int64_t n, int slice_rows,
                                         float* __restrict__ part,
                                         float* __restrict__ ynorm_part, int64_t j0, int s,
                                         int k0, bool write_ynorm,
                                         const uint4* __restrict__ Csp, int64_t ldq) {
    static_assert(NKB >= 1 && NKB <= kKC / 16, "group blocks per tile");
    constexpr size_t kCBuf = 2 * kKC * kStrideH * sizeof(__bf16);   // hi and lo of one stage
    __shared__ __attribute__((aligned(16))) char smem[2 * kCBuf];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    __syncthreads();   // a previous tile of this workgroup may still read the LDS
    const int q = lane & 15, g = lane >> 4;
    const int64_t r0 = (int64_t)s * slice_rows;
    const int64_t r1 = r0 + slice_rows < d ? r0 + slice_rows : d;
    const int nkb = (kpad - k0 < kKC ? kpad - k0 : kKC) / 16;   // blocks written out

    floatx4 acc[2][NKB];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NKB; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    float ycol[2] = {0.f, 0.f};   // this lane's share of its two columns' squared norms

    // this lane's two columns (clamped into the matrix: their outputs are dropped)
    const float* yp[2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        int64_t col = j0 + wave * 32 + jb * 16 + q;
        if (col >= n) col = n - 1;
        yp[jb] = Y + col * ldy + 4 * g;
    }
    static_assert(AHEAD == 1 || AHEAD == 2, "stages in flight");
    float4 ya[2][2], yb[2][2];   // [jb][half]: column values of stage r and (AHEAD 2) r + kRT
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int h = 0; h < 2; ++h) yb[jb][h] = make_float4(0.f, 0.f, 0.f, 0.f);
    SplitStage<64 * WAVES, 16 * NKB> rs;   // only the groups the MFMAs read
    rs.init(Csp, ldq, k0, kpad);
    // a stage inside the rows: unconditional loads
    auto load_y_full = [&](int64_t r, float4 (&yv)[2][2]) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int h = 0; h < 2; ++h) yv[jb][h] = *reinterpret_cast<const float4*>(yp[jb] + r + 16 * h);
    };
    // any stage: rows past r1 read row 0 of the column and are zeroed
    auto load_y_any = [&](int64_t r, float4 (&yv)[2][2]) {
        if (r + kRT <= r1) {
            load_y_full(r, yv);
            return;
        }
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bool in = r + 4 * g + 16 * h < r1;
                const float4 t = *reinterpret_cast<const float4*>(in ? yp[jb] + r + 16 * h : yp[jb] - 4 * g);
                yv[jb][h] = in ? t : make_float4(0.f, 0.f, 0.f, 0.f);
            }
    };
    auto store_c = [&](int b) {
        __bf16* Ch = reinterpret_cast<__bf16*>(smem + b * kCBuf);
        rs.template store<true>(Ch, Ch + kKC * kStrideH);
    };
    // the loaded column values as A operands (and their squares)
    auto split = [&](const float4 (&yv)[2][2], bf16x8 (&ahi)[2], bf16x8 (&alo)[2]) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            const float x[8] = {yv[jb][0].x, yv[jb][0].y, yv[jb][0].z, yv[jb][0].w,
                                yv[jb][1].x, yv[jb][1].y, yv[jb][1].z, yv[jb][1].w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 h = (__bf16)x[e];
                ahi[jb][e] = h;
                alo[jb][e] = (__bf16)(x[e] - (float)h);
                ycol[jb] += x[e] * x[e];
            }
        }
    };
    auto mfma_stage = [&](int b, const bf16x8 (&ahi)[2], const bf16x8 (&alo)[2]) {
        const __bf16* Ch = reinterpret_cast<const __bf16*>(smem + b * kCBuf);
        const __bf16* Cl = Ch + kKC * kStrideH;
        bf16x8 bhi[NKB], blo[NKB];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            const int row = kb * 16 + q;
            bhi[kb] = *reinterpret_cast<const bf16x8*>(Ch + row * kStrideH + g * 8);
            blo[kb] = *reinterpret_cast<const bf16x8*>(Cl + row * kStrideH + g * 8);
        }
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
                acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[jb], bhi[kb], acc[jb][kb], 0, 0, 0);
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
                acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[jb], blo[kb], acc[jb][kb], 0, 0, 0);
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
                acc[jb][kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[jb], bhi[kb], acc[jb][kb], 0, 0, 0);
    };
    auto copy_y = [&](float4 (&dst)[2][2], const float4 (&src)[2][2]) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int h = 0; h < 2; ++h) dst[jb][h] = src[jb][h];
    };
    bf16x8 ahi[2], alo[2];
    int b = 0;
    int64_t r = r0;
    if constexpr (AHEAD == 1) {
        // At the top of each pass LDS buffer b holds the centroids of stage r and
        // ya its column values; the next stage's loads run during the MFMAs.
        if (r0 < r1) {
            load_y_any(r0, ya);
            rs.load_rows(r0);
            store_c(0);
            __syncthreads();
        }
        for (; r + 2 * kRT <= r1; r += kRT, b ^= 1) {   // the next stage lies inside the rows
            split(ya, ahi, alo);
            load_y_full(r + kRT, ya);
            rs.load_rows(r + kRT);
            mfma_stage(b, ahi, alo);
            store_c(b ^ 1);
            __syncthreads();
        }
        for (; r < r1; r += kRT, b ^= 1) {              // the last stage (or the next one partial)
            split(ya, ahi, alo);
            const bool more = r + kRT < r1;
            if (more) {
                load_y_any(r + kRT, ya);
                rs.load_rows(r + kRT);
            }
            mfma_stage(b, ahi, alo);
            if (more) store_c(b ^ 1);
            __syncthreads();
        }
    } else {
        // Loads complete in issue order, so a step issues the centroids and the
        // column values of stage r + 2 kRT together: waiting for the centroids of
        // stage r + kRT (loaded a step earlier) then leaves both later stages in
        // flight.  At the top of each pass LDS buffer b holds the centroids of stage
        // r, ya (or yb) the column values of stage r and the other set those of
        // stage r + kRT, and rsb (or rsa) the centroids of stage r + kRT.
        SplitStage<64 * WAVES, 16 * NKB> rsb = rs;
        if (r0 < r1) {
            rs.load_rows(r0);
            load_y_any(r0, ya);
            if (r0 + kRT < r1) {
                rsb.load_rows(r0 + kRT);
                load_y_any(r0 + kRT, yb);
            }
            store_c(0);
            __syncthreads();
        }
        auto store_from = [&](const SplitStage<64 * WAVES, 16 * NKB>& src, int bb) {
            __bf16* Ch = reinterpret_cast<__bf16*>(smem + bb * kCBuf);
            src.template store<true>(Ch, Ch + kKC * kStrideH);
        };
        // stages up to r + 2 kRT inside the rows
        auto step = [&](float4 (&cur)[2][2], SplitStage<64 * WAVES, 16 * NKB>& ld,
                        const SplitStage<64 * WAVES, 16 * NKB>& st) {
            // (the barriers keep each stage's work in its own step: hoisting the next
            // stage's split here would wait on values still in flight)
            __builtin_amdgcn_sched_barrier(0);
            split(cur, ahi, alo);
            __builtin_amdgcn_sched_barrier(0);
            ld.load_rows(r + 2 * kRT);
            load_y_full(r + 2 * kRT, cur);
            __builtin_amdgcn_sched_barrier(0);
            mfma_stage(b, ahi, alo);
            store_from(st, b ^ 1);
            __syncthreads();
            r += kRT;
            b ^= 1;
        };
        for (; r + 4 * kRT <= r1;) {   // two steps per pass: the sets trade roles in place
            step(ya, rs, rsb);
            step(yb, rsb, rs);
        }
        if (r + 3 * kRT <= r1) {   // one more whole step leaves stage r in yb: swap the sets
            step(ya, rs, rsb);
            float4 t[2][2];
            copy_y(t, ya);
            copy_y(ya, yb);
            copy_y(yb, t);
            const SplitStage<64 * WAVES, 16 * NKB> u = rs;
            rs = rsb;
            rsb = u;
        }
        for (; r < r1; r += kRT, b ^= 1) {   // at most three stages left
            split(ya, ahi, alo);
            const bool more = r + kRT < r1;
            copy_y(ya, yb);
            if (r + 2 * kRT < r1) {
                rs.load_rows(r + 2 * kRT);
                load_y_any(r + 2 * kRT, yb);
            }
            mfma_stage(b, ahi, alo);
            if (more) store_from(rsb, b ^ 1);
            __syncthreads();
            rsb = rs;
        }
    }
    if (write_ynorm) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            float t = ycol[jb];
            t += __shfl_xor(t, 16);
            t += __shfl_xor(t, 32);
            const int64_t j = j0 + wave * 32 + jb * 16 + q;
            if (g == 0 && j < n) ynorm_part[(int64_t)s * n + j] = t;
        }
    }
    // lane holds D[column 4g + v][group q] of each 16 x 16 tile
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            if (kb >= nkb) continue;
            const int k = k0 + kb * 16 + q;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t j = j0 + wave * 32 + jb * 16 + 4 * g + v;
                if (j < n) part[((int64_t)s * n + j) * kpad + k] = acc[jb][kb][v];
            }
        }
}


// dot[t] = sum over the slices, in slice order, of part[s][j][q + 16 t] (zero for
// groups >= c; q may include a group offset), and (YN) ynorm = the same sum of
// ynorm_part[s][j].
// Four slices' loads are issued before their additions; the loads are
// unconditional (indices clamped into the buffer, unwanted values zeroed after
// the load) so that they are not serialised behind branches.
template <int T, bool YN>
__device__ inline void sum_slices(const float* __restrict__ part,
                                  const float* __restrict__ ynorm_part, int nslices, int64_t n,
                                  int64_t j, int c, int kpad, int q, double (&dot)[T],
                                  double& ynorm) {
#pragma unroll
    for (int t = 0; t < T; ++t) dot[t] = 0.0;
    ynorm = 0.0;
    for (int s = 0; s < nslices; s += 4) {
        float v[4][T], yn[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int su = s + u < nslices ? s + u : nslices - 1;
            const float* p = part + ((int64_t)su * n + j) * kpad;
#pragma unroll
            for (int t = 0; t < T; ++t) v[u][t] = p[q + 16 * t < kpad ? q + 16 * t : kpad - 1];
            yn[u] = YN ? ynorm_part[(int64_t)su * n + j] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = s + u < nslices;
#pragma unroll
            for (int t = 0; t < T; ++t) dot[t] += (ok && q + 16 * t < c) ? (double)v[u][t] : 0.0;
            ynorm += ok ? (double)yn[u] : 0.0;
        }
    }
}


}  // namespace respca
