// Internal launchers of librespca's gfx950 kernels.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace respca {

constexpr int kBlock = 256;          // threads of a streaming workgroup (4 wave64)
constexpr int kRowsPerBlock = 1024;  // rows of the d-slice one streaming workgroup covers
constexpr int kSegCols = 64;         // max columns of one group segment in the means pass
constexpr int kMaxGroups = 1024;     // c limit (LDS histogram of the label sort)
constexpr int kPickThreads = 1024;   // single-workgroup k-means++ draw

inline int row_blocks(int64_t d) { return (int)((d + kRowsPerBlock - 1) / kRowsPerBlock); }
inline int max_segments(int64_t n, int c) { return (int)((n + kSegCols - 1) / kSegCols) + c; }

// Fill a d x n column-major array (leading dimension ld) with zeros.
template <typename T>
void launch_zero2d(T* A, int64_t ld, int64_t d, int64_t n, hipStream_t st);
void launch_zero_i32(int32_t* a, int64_t count, hipStream_t st);
void launch_zero_f64(double* a, hipStream_t st);

// Sum of squares of X in double: per-workgroup partials, count returned.
template <typename T>
int launch_sumsq(const T* X, int64_t ldx, int64_t d, int64_t n, double* partial, hipStream_t st);
// Fixed-order sum of `count` partial triples/singles into out[0..width).
void launch_sum_partials(const double* partial, int count, int width, double* out, hipStream_t st);

// Stable counting sort of labels: counts[c], perm[n] (columns grouped by label,
// increasing index within a group), and the segment table of the means pass.
// `bc` is scratch of sort_scratch_ints(n, c) ints.
int64_t sort_scratch_ints(int64_t n, int c);
void launch_label_sort(const int32_t* labels, int64_t n, int c, int32_t* bc, int32_t* counts,
                       int32_t* perm, int32_t* seg_begin, int32_t* seg_len, int32_t* seg_first,
                       int32_t* nseg, hipStream_t st);

// Group partial sums: partial[s*d + i] = sum over the columns j of segment s of
// Y[i, j], where Y = X - S + Theta*inv_rho (with_d = true) or Y = A (with_d = false).
template <typename T>
void launch_group_partial(bool with_d, const T* A, int64_t lda, const T* S, int64_t lds,
                          const T* Th, int64_t ldt, T inv_rho, int64_t d, int64_t n, int c,
                          const int32_t* perm, const int32_t* seg_begin, const int32_t* seg_len,
                          const int32_t* nseg, double* partial, hipStream_t st, int max_seg = -1);

// C[:, k] = (sum of the segment partials of group k) / n_k for non-empty groups;
// with gsum, also gsum[:, k] = that sum in double (zero for empty groups).
template <typename T>
void launch_group_finalize(const double* partial, int64_t d, int c, const int32_t* counts,
                           const int32_t* seg_first, T* C, hipStream_t st, double* gsum = nullptr);

// Incremental group means after an assignment pass (see kernels.hip): a
// counting sort of the moved columns under 2c keys (entering new label, leaving
// old label), the new group counts, and its segment table; then, after the
// group partials of those segments, the update of the group sums and means.
// `bc` holds changed_sort_scratch_ints(n, c) ints; perm 2n entries; seg_begin and
// seg_len max_seg entries (enough: changed_max_segments(moved, c)), seg_first
// 2c + 1.
int64_t changed_sort_scratch_ints(int64_t n, int c);
int changed_max_segments(int64_t moved, int c);
void launch_changed_sort(const int32_t* new_labels, const int32_t* old_labels, int64_t n, int c,
                         int32_t* bc, const int32_t* counts_old, int32_t* counts_new, int32_t* perm,
                         int32_t* seg_begin, int32_t* seg_len, int32_t* seg_first, int32_t* nseg,
                         int max_seg, hipStream_t st);
// The update also copies counts_new to counts_out (the group counts the next
// pass starts from).
template <typename T>
void launch_group_update(const double* partial, int64_t d, int c, const int32_t* counts_new,
                         const int32_t* seg_first, double* gsum, T* C, int32_t* counts_out,
                         hipStream_t st);

// out[k] = ||C[:, k]||^2 in double.
template <typename T>
void launch_col_sqnorm(const T* C, int64_t d, int c, double* out, hipStream_t st);

// One ALM sweep over every entry: L-step, S-step, multiplier update, and the
// three squared-norm partials (returns the number of partial triples).
// The sweep walked in group order (segments of the last label sort); also writes
// the group partial sums of D' = X - S' + Theta' * inv_rho_next to next_partial
// (layout of the means pass).  Returns the number of norm partials (slots past
// the segment count contribute zeros).
int sweep_seg_partials(int64_t d, int64_t n, int c);
template <typename T>
int launch_sweep_seg(const T* X, int64_t ldx, T* L, int64_t ldl, T* S, int64_t lds, T* Th,
                     int64_t ldt, const T* C, const int32_t* labels, const int32_t* perm,
                     const int32_t* seg_begin, const int32_t* seg_len, const int32_t* nseg,
                     int64_t d, int64_t n, int c, double alpha, double beta, double rho,
                     double inv_rho, double inv_rho_next, double* norm_partial,
                     double* next_partial, hipStream_t st, const double* l21_fac = nullptr);

// Column-wise (l2,1) S-step factors: fac[j] = max(0, 1 - 1/(rho ||B_j||)) with
// B = X - L + Theta * inv_rho and L the L-step's alpha D + beta C[:, labels[j]]
// (D = X - S + Theta * inv_rho), evaluated as the sweep evaluates it.  Passing
// fac to launch_sweep_seg then makes its S-step S_j = fac[j] B_j.
// The l1 sweep on the compact state: B (d x n, ldb) holds X - L + Theta/rho of
// the previous iteration (penalty rho_prev), from which S = soft(B, 1/rho_prev)
// and Theta = clip(rho_prev B); reads X, B, L and writes L and the new B.  Same
// norm partials, next-step group sums and grid as launch_sweep_seg.
template <typename T>
int launch_sweep_seg_compact(const T* X, int64_t ldx, T* L, int64_t ldl, T* B, int64_t ldb,
                             const T* C, const int32_t* labels, const int32_t* perm,
                             const int32_t* seg_begin, const int32_t* seg_len, const int32_t* nseg,
                             int64_t d, int64_t n, int c, double alpha, double beta, double rho,
                             double inv_rho, double inv_rho_next, double rho_prev,
                             double inv_rho_prev, double* norm_partial, double* next_partial,
                             hipStream_t st);

// Group partial sums of D = X - S + Theta inv_rho from the compact state (as
// launch_group_partial with with_d).
template <typename T>
void launch_group_partial_compact(const T* X, int64_t ldx, const T* B, int64_t ldb, T inv_rho,
                                  T rho_prev, T inv_rho_prev, int64_t d, int64_t n, int c,
                                  const int32_t* perm, const int32_t* seg_begin,
                                  const int32_t* seg_len, const int32_t* nseg, double* partial,
                                  hipStream_t st);

// B <- soft(B, tau) in place (the S of a compact state).
template <typename T>
void launch_soft_inplace(T* B, int64_t ldb, int64_t d, int64_t n, double tau, hipStream_t st);

template <typename T>
void launch_l21_factor(const T* X, int64_t ldx, const T* S, int64_t lds, const T* Th, int64_t ldt,
                       const T* C, const int32_t* labels, int64_t d, int64_t n, double alpha,
                       double beta, double rho, double inv_rho, double* fac, hipStream_t st);


// Split-d centroid/column dot products: part[(rb*c + k)*n + j] = sum_{i in slice rb} C[i,k] Y[i,j],
// over dots_slices(d, n, c) slices of dots_slice_rows(d, n, c) rows (whole 32-row
// stages, at most kRowsPerBlock; short slices when the column tiles alone would
// leave the GPU idle).
int64_t dots_slice_rows(int64_t d, int64_t n, int c);
int dots_slices(int64_t d, int64_t n, int c);
template <typename T>
void launch_dots(const T* C, int64_t d, int c, const T* Y, int64_t ldy, int64_t n, T* part,
                 hipStream_t st);

// labels_new[j] = argmin_k ||C_k||^2 - 2 C_k . Y_j (ties: lowest k); per-block
// counts of changed labels.  Returns the number of count partials.
template <typename T>
int launch_argmin(const T* part, int nrb, int c, int64_t n, const double* cnorm,
                  const int32_t* old_labels, int32_t* new_labels, double* changed_partial,
                  hipStream_t st);

// Assignment pass: new_labels[j] = argmin_k ||C_k||^2 - 2 C_k . Y_j (ties: lowest
// k), per-block changed counts into changed_partial; returns the number of
// count partials.  `work` must hold assign_workspace_bytes<T>(d, n, c).
template <typename T>
size_t assign_workspace_bytes(int64_t d, int64_t n, int c);
// bf16 (float runs only): labels of the FP64 distances of the FP32 values.  Above
// 16 groups a bounded-error MFMA contraction (split-bf16, or FP32 up to 32 groups)
// with exact refinement of near-tied columns, whose changes are counted in the int
// at assign_refine_counters(work)[1] (*changed_extra is set to 1 when that
// applies); at most 16 groups an FP64 contraction with nothing to refine.
// cnorm (||C_k||^2 in double) is an input, except in bf16 mode, where the pass
// computes it while splitting the centroids.
template <typename T>
int launch_assign(const T* C, int64_t d, int c, const T* Y, int64_t ldy, int64_t n,
                  double* cnorm, const int32_t* old_labels, int32_t* new_labels, void* work,
                  double* changed_partial, bool bf16, int* changed_extra, hipStream_t st);
int* assign_refine_counters(void* work, int64_t d, int64_t n, int c);
// out[0] += counter (or out[0] = counter when set), one thread.
// Status words a finishing kernel can also hand to the host: the five device
// words `words` (norms, changed count, refined count) are copied to the pinned
// host words `host`, then, after a system-scope fence, `seq` goes to `host_seq`.
// seq == 0: nothing is published.
struct StatusPublish {
    const double* words = nullptr;
    double* host = nullptr;
    uint64_t* host_seq = nullptr;
    uint64_t seq = 0;
};
// out[0] = sum of `count` changed-count partials plus counters[1]; out[1] =
// counters[0] (counters may be null: refinement counts then read as zero).  With
// pub.seq set (pub.words + 3 == out), the words are published with out[0..1] as
// computed here, and out[1] is left at zero so the refined count is taken once.
void launch_assign_finish(const double* partial, int count, const int* counters, double* out,
                          hipStream_t st, const StatusPublish& pub = StatusPublish());
void launch_add_int(const int* counter, double* out, hipStream_t st, bool set = false);
inline int64_t assign_partials_max(int64_t n) { return (n + 15) / 16; }

// k-means++ helpers.
template <typename T>
void launch_d2(const T* Y, int64_t ldy, int64_t d, int64_t n, const int32_t* seeds, int m,
               double* d2, hipStream_t st);
// Bounded k-means++ seeding for float runs: launch_d2_first does the m = 0
// pass and fills the fp16 copy Z (d2_copy_ld(d) rows per column), its column
// scales zsc[n] and the column norms ynorm[n]; launch_d2_bounded then does pass
// m >= 1 with the same results as launch_d2.
int64_t d2_copy_ld(int64_t d);
void launch_d2_first(const float* Y, int64_t ldy, int64_t d, int64_t n, const int32_t* seeds,
                     double* d2, _Float16* Z, float* zsc, double* ynorm, hipStream_t st);
void launch_d2_bounded(const float* Y, int64_t ldy, int64_t d, int64_t n, const int32_t* seeds,
                       int m, double* d2, const _Float16* Z, const float* zsc, const double* ynorm,
                       hipStream_t st);
void launch_pick(const double* d2, int64_t n, const double* u, int m, int32_t* seeds,
                 int32_t* chosen, hipStream_t st);
template <typename T>
void launch_gather_cols(const T* Y, int64_t ldy, int64_t d, const int32_t* idx, int c, T* C,
                        hipStream_t st);

}  // namespace respca
