/*
 * respca.h -- C ABI of librespca, an MI355X (gfx950) implementation of RES-PCA
 * (Peng et al., "RES-PCA: A Scalable Approach to Recovering Low-rank Matrices",
 * arXiv 1904.07497).
 *
 * Problem (Sec. 3, eq. eq_obj): split a d x n matrix X into L + S, where the
 * columns of L are pulled toward the means of c groups (the within-group
 * variance term, weight lambda) and S is sparse (l1 norm), the groups being
 * learned by K-means.  Solved by the ALM iteration of Sec. 4: an L-step in
 * closed form (Sec. 4.1), a p-step by K-means on the columns of L (Sec. 4.2), a
 * soft-threshold S-step (Sec. 4.3) and the multiplier/penalty update (Sec. 4.4),
 * stopped by the rule of Sec. 5.
 *
 * Conventions shared by every call
 *   - Matrices are column-major (BLAS convention): entry (i, j) of an array
 *     with leading dimension ld is at ptr[j*ld + i]; column j is sample j.
 *     Leading dimensions must be >= d.
 *   - Matrix and label pointers are DEVICE pointers on the handle's device
 *     unless a comment says "host".  Element type: double for RESPCA_F64,
 *     float for RESPCA_F32 and RESPCA_BF16GEMM_F32.
 *   - The caller owns every buffer passed in; the library keeps no pointer
 *     after a call returns.  X is read-only.  L, S, Theta, X must not overlap.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  All work
 *     is enqueued on it; calls that return an info struct block until it is
 *     complete (they read a few bytes back per iteration).
 *   - Errors are reported only by the return code; no call throws or aborts.
 *     On an error (< 0) the outputs are unspecified; respca_last_error()
 *     gives a message.  Calls on one handle must not overlap in time.
 *   - Limits: 1 <= c <= min(n, 1024); d, n < 2^31.
 */
#ifndef RESPCA_H
#define RESPCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RESPCA_OK = 0,               /* converged (criterion <= tol)                      */
    RESPCA_NOT_CONVERGED = 1,    /* max_iter reached; outputs are the last iterate    */
    RESPCA_ERR_INVALID = -1,     /* bad size, parameter, pointer or aliasing          */
    RESPCA_ERR_NONFINITE = -2,   /* X holds NaN or Inf (found by the ||X||_F pass)    */
    RESPCA_ERR_NOMEM = -3,       /* device allocation failed                          */
    RESPCA_ERR_HIP = -4,         /* a HIP runtime call failed                         */
    RESPCA_ERR_UNSUPPORTED = -5  /* valid request outside this build's limits         */
} respca_status;

typedef enum {
    RESPCA_F64 = 0,              /* everything in double                              */
    RESPCA_F32 = 1,              /* float data and arithmetic, double accumulators    */
    RESPCA_BF16GEMM_F32 = 2      /* as F32, but K-means labels from FP64 distances of
                                    the FP32 values: above 32 groups split-bf16 MFMA
                                    with bounds and an exact re-check of close calls,
                                    17-32 groups FP32 MFMA with bounds and the same
                                    re-check, at most 16 groups FP64 dot products    */
} respca_precision;

/* Penalty on the sparse term S.  L1 is the entrywise l1 norm of eq_obj (Sec. 3;
 * S-step of Sec. 4.3: entrywise soft threshold at 1/rho).  L21 is the column-wise
 * l2,1 norm named after eq_obj as the alternative (norm of eq_rpca_l21, Sec. 2):
 * the S-step becomes S_j = B_j max(0, 1 - 1/(rho ||B_j||_2)) per column j, with
 * B = X - L + Theta/rho, and needs one extra read of X, S and Theta per iteration
 * for the column norms.  The solver and iterate entry points take both; the
 * batched solver takes L1 only (RESPCA_ERR_UNSUPPORTED otherwise). */
typedef enum {
    RESPCA_SPARSE_L1 = 0,
    RESPCA_SPARSE_L21 = 1
} respca_sparse_norm;

/* How the p-step finds the groups.  KMEANS is the method of Sec. 4.2: Lloyd's
 * passes on the columns of L from the current groups.  SPECTRAL is the nonlinear
 * alternative the end of Sec. 4.2 names (and the Remark closing Sec. 3): normalised
 * spectral clustering (Ng, Jordan & Weiss 2001) of the columns of L with the
 * Gaussian affinity W_ij = exp(-||L_i - L_j||^2 / (2 sigma^2)), W_ii = 0,
 * A = D^{-1/2} W D^{-1/2}, rows of the eigenvectors of the c largest eigenvalues
 * scaled to unit length, then Lloyd's passes on those rows from the current groups
 * (centroids = group means of the rows, an empty group at zero).  The initial
 * groups are the spectral clustering of X's columns with k-means++ seeding from
 * `seed` then Lloyd.  L-, S- and multiplier steps are unchanged.  It holds the
 * n x n affinity in FP64 (8 n^2 bytes): n <= 32768 and c <= 40, else
 * RESPCA_ERR_UNSUPPORTED; solve and iterate only (batched, no-alloc and
 * init_embedding: RESPCA_ERR_UNSUPPORTED). */
typedef enum {
    RESPCA_PSTEP_KMEANS = 0,
    RESPCA_PSTEP_SPECTRAL = 1
} respca_pstep;

typedef struct {
    double   lambda;      /* weight of the group-variance term of eq_obj (Sec. 3); must be
                             >= 0.  NaN selects sqrt(max(d, n)), the value of Sec. 5.1.   */
    int32_t  rank;        /* c, the number of groups; 0 selects 5 (Sec. 5.1, unknown rank) */
    double   tol;         /* stopping tolerance of the Sec. 5 criterion; default 1e-3      */
    int32_t  max_iter;    /* outer-iteration cap; default 500 (Sec. 5)                      */
    double   rho0;        /* initial penalty; default 1e-4 (Sec. 5.1)                       */
    double   kappa;       /* penalty growth factor, > 1; default 1.5 (Sec. 4.4, 5.1)        */
    double   rho_max;     /* cap on rho (not in the paper); default 1e10                    */
    int32_t  max_lloyd;   /* cap on Lloyd assignment passes per K-means call; default 100   */
    uint64_t seed;        /* splitmix64 seed of the k-means++ initialisation; default 0     */
    int32_t  precision;   /* respca_precision; default RESPCA_F32                           */
    const int32_t *init_labels; /* optional device int32[n] in [0, c): initial groups used
                             instead of k-means++ + Lloyd on X (warm start); NULL = none   */
    double  *history;     /* optional HOST double[3 * max_iter]: per iteration the three
                             relative criterion terms (primal, dL, dS); NULL = none        */
    const void *init_embedding; /* optional device FP32 matrix, init_embedding_rows x n with
                             leading dimension init_embedding_ld: its columns are clustered
                             (k-means++ from seed, then Lloyd) in place of the seeding on X;
                             from the means of X over those groups (empty groups at zero)
                             Lloyd then runs on the columns of X (same rule as the p-step,
                             at most max_lloyd passes), and the iterations start as with
                             init_labels from the resulting groups.  info.init_lloyd counts
                             the passes of both.  Ignored when init_labels is set; not for
                             RESPCA_F64.  NULL = none                                       */
    int64_t  init_embedding_ld;
    int32_t  init_embedding_rows;
    int32_t  sparse_norm; /* respca_sparse_norm; default RESPCA_SPARSE_L1; other values
                             RESPCA_ERR_INVALID                                             */
    int32_t  pstep;       /* respca_pstep; default RESPCA_PSTEP_KMEANS                      */
    double   spectral_sigma; /* kernel width of the spectral p-step (the paper gives none):
                             > 0 the width sigma itself; < 0 relative, sigma = |value| times
                             the RMS distance of the clustered columns to their mean column
                             (follows the scale of L, which the L-step shrinks toward the
                             group means in early iterations); 0 or non-finite
                             RESPCA_ERR_INVALID with the spectral p-step; default 0        */
    int32_t  init_embedding_refine; /* with init_embedding: 1 (default) runs the Lloyd passes
                             on X after the embedding's K-means, 0 starts the iterations
                             from the embedding's groups directly, 2 uses the embedding
                             for the k-means++ seeding only (distances between embedding
                             columns place the c seeds; the seed columns of X then start
                             the nearest-seed assignment and Lloyd on X, as without an
                             embedding); other values RESPCA_ERR_INVALID                   */
} respca_params;

typedef struct {
    int32_t iters;        /* outer iterations run                                       */
    int32_t lloyd_steps;  /* assignment passes summed over the outer iterations         */
    int32_t init_lloyd;   /* assignment passes of the initial K-means on X              */
    int32_t status;       /* respca_status of the call                                  */
    double  primal;       /* ||X - L - S||_F / ||X||_F at the last iteration            */
    double  dL;           /* ||L_t - L_{t-1}||_F / ||X||_F                              */
    double  dS;           /* ||S_t - S_{t-1}||_F / ||X||_F                              */
    double  rho_final;    /* rho used by the last iteration                             */
    int64_t refined;      /* bf16 mode: column decisions re-taken exactly (all passes;
                             zero at most 16 groups, where nothing is re-taken)          */
    int32_t eig_iters;    /* spectral p-step: filtered subspace iterations, all p-steps  */
    int32_t eig_unconverged; /* spectral p-step: embeddings whose eigen residual stayed
                             above 1e-10 after 100 iterations                            */
} respca_info;

typedef struct respca_handle_s *respca_handle;

/* Create a handle bound to HIP device `device` (its workspace grows on demand
 * and is freed by respca_destroy).  Returns RESPCA_ERR_HIP if the device is
 * unavailable. */
respca_status respca_create(respca_handle *out, int32_t device);
void          respca_destroy(respca_handle h);

/* Fill *p with the defaults listed above.  Needs no device. */
void          respca_params_default(respca_params *p);
/* Static strings.  Need no device. */
const char   *respca_status_string(respca_status s);
const char   *respca_last_error(respca_handle h);
/* Version string of the library build.  Needs no device. */
const char   *respca_version(void);

/*
 * Whole solve (Sec. 4 iteration with the Sec. 5 stopping rule).
 *   X (d x n, ldx), read-only.  L (d x n, ldl) and S (d x n, lds) receive the
 *   low-rank and sparse parts.  labels (nullable, device int32[n]) receives the
 *   final groups.  info (host, nullable) receives the counters.
 * Initialisation (not specified by the paper): S = Theta = 0, L_0 = 0,
 * rho = rho0, groups = K-means of the columns of X (k-means++ seeding from
 * splitmix64(seed), then Lloyd) unless params->init_labels is given.
 * ||X||_F == 0 returns RESPCA_OK with L = S = 0, labels 0 and iters = 0.
 * With the l1 penalty, S also holds the iteration's working state (X - L +
 * Theta/rho, from which the S-step and the multiplier follow) and receives the
 * sparse part when the iterations end.
 * Returns RESPCA_OK, RESPCA_NOT_CONVERGED or an error (then L and S are
 * unspecified).
 */
respca_status respca_solve(respca_handle h, const respca_params *params,
                           int64_t d, int64_t n,
                           const void *X, int64_t ldx,
                           void *L, int64_t ldl,
                           void *S, int64_t lds,
                           int32_t *labels, respca_info *info, void *stream);

/*
 * Run `iters` outer iterations (Sec. 4.1 -> 4.2 -> 4.3 -> 4.4) from a state the
 * caller holds, updating it in place; no initialisation and no stopping test.
 *   L (ldl): on entry L_{t-1}, on exit L_t.   S (lds), Theta (ldt): previous ->
 *   new iterate.   labels (device int32[n]) and C (device d x c, leading
 *   dimension d: group centroids, used for groups that are empty) in/out.
 *   *rho (host): rho_t on entry, the next rho on exit.
 *   norms (host, nullable): 3 doubles per iteration, the absolute Frobenius
 *   norms ||X-L-S||, ||L_t-L_{t-1}||, ||S_t-S_{t-1}||.
 * This is the checkpoint/resume and step-by-step interface.
 */
respca_status respca_iterate(respca_handle h, const respca_params *params,
                             int64_t d, int64_t n,
                             const void *X, int64_t ldx,
                             void *L, int64_t ldl,
                             void *S, int64_t lds,
                             void *Theta, int64_t ldt,
                             int32_t *labels, void *C, double *rho, int32_t iters,
                             double *norms, respca_info *info, void *stream);

/*
 * respca_iterate without device allocation, for callers that cannot allocate
 * (code running between graph captures, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and error codes are those of
 * respca_iterate; its workspace (label sort tables, group partial sums,
 * distance partials, Lloyd's moved-column tables, status words) comes from a
 * fixed device array of RESPCA_NOALLOC_SCRATCH_BYTES per GPU, held by the
 * library until the process ends, instead of the handle.  A problem whose
 * workspace would exceed it returns RESPCA_ERR_UNSUPPORTED before any work is
 * enqueued (respca_last_error gives the bytes needed).  The call does not time
 * kernels (respca_profile_enable has no effect on it).  Every call on one GPU,
 * from any handle, uses that GPU's single array and leaves its contents behind:
 * calls that overlap in time on one GPU race and must be serialised by the
 * caller.
 */
#define RESPCA_NOALLOC_SCRATCH_BYTES (64u << 20)
respca_status respca_iterate_noalloc(respca_handle h, const respca_params *params,
                                     int64_t d, int64_t n,
                                     const void *X, int64_t ldx,
                                     void *L, int64_t ldl,
                                     void *S, int64_t lds,
                                     void *Theta, int64_t ldt,
                                     int32_t *labels, void *C, double *rho, int32_t iters,
                                     double *norms, respca_info *info, void *stream);

/*
 * K-means of the columns of Y (d x n, ldy): k-means++ seeding driven by
 * splitmix64(params->seed), nearest-seed assignment, group means (an empty group
 * keeps its seed), then Lloyd passes until no label changes or max_lloyd.
 * labels (device int32[n]) and C (device d x c, leading dimension d) are
 * outputs; info->init_lloyd receives the number of Lloyd passes.  This is the
 * initialisation respca_solve uses (the p-step of Sec. 4.2 applied to X).
 */
respca_status respca_kmeans(respca_handle h, const respca_params *params,
                            int64_t d, int64_t n, const void *Y, int64_t ldy,
                            int32_t *labels, void *C, respca_info *info, void *stream);

/*
 * Row embedding of the spectral p-step on its own (RESPCA_PSTEP_SPECTRAL): for
 * the columns of Y (d x n, ldy; double if precision is RESPCA_F64, else float)
 * emb (device, c x n doubles, leading dimension c) receives the unit rows of
 * the eigenvectors of the c largest eigenvalues of D^{-1/2} W D^{-1/2},
 * W_ij = exp(-||Y_i - Y_j||^2 / (2 s^2)), W_ii = 0, s = sigma for sigma > 0 and
 * |sigma| times the RMS distance of the columns to their mean for sigma < 0
 * (sigma = 0 or non-finite: RESPCA_ERR_INVALID) (any orthonormal basis of
 * that eigenspace: K-means of the rows depends only on their distances).
 * eigenvalues (host, nullable) receives the c largest eigenvalues (decreasing),
 * info (host, nullable) eig_iters / eig_unconverged.  Limits as for the p-step.
 */
respca_status respca_spectral_embedding(respca_handle h, int32_t precision, int64_t d, int64_t n,
                                        const void *Y, int64_t ldy, int32_t c, double sigma,
                                        uint64_t seed, double *emb, double *eigenvalues,
                                        respca_info *info, void *stream);

/*
 * Anomaly scores (Sec. 5.3, the anomaly-detection experiment: the columns of the
 * recovered S with a large l2 norm are the outlying samples): out[j] = ||S_j||_2
 * for the n columns of S (d x n, leading dimension lds >= max(d, 1); double if
 * precision is RESPCA_F64, else float), summed in double in a fixed order.  out:
 * device, n doubles, written on `stream`.  d = 0 gives zeros; n = 0 does
 * nothing.  RESPCA_ERR_INVALID for a bad precision, negative sizes, lds < d or a
 * null pointer with d, n > 0.  The threshold that separates outliers is the
 * caller's (the paper blanks scores below 5 on its data).
 */
respca_status respca_column_norms(respca_handle h, int32_t precision, int64_t d, int64_t n,
                                  const void *S, int64_t lds, double *out, void *stream);

/*
 * Batched solve: `batch` independent RES-PCA problems of uneven size, each run
 * exactly as respca_solve would run it (its own initial K-means, iteration
 * count, Lloyd passes and Sec. 5 stopping test), all inside one persistent
 * kernel launch that is captured once in a hipGraph and replayed when the same
 * call (same pointers, sizes and parameters) repeats.
 *   params[i]: per-instance parameters (precision must be RESPCA_F32; the
 *              history pointer is ignored).  d[i], n[i], ldx[i], ldl[i], lds[i]:
 *              sizes and leading dimensions.  X[i], L[i], S[i]: device pointers
 *              (host arrays of them).  labels: nullable host array of nullable
 *              device int32[n[i]] pointers.  info: host array of `batch` structs.
 * Tile shapes come from the handle's tuning (respca_autotune_batched) or the
 * defaults.  At most 1024 instances per call (RESPCA_ERR_UNSUPPORTED beyond).  Returns RESPCA_OK when every instance converged, otherwise the
 * first non-OK instance status (each info[i].status has its own).
 */
respca_status respca_solve_batched(respca_handle h, const respca_params *params, int32_t batch,
                                   const int64_t *d, const int64_t *n,
                                   const void *const *X, const int64_t *ldx,
                                   void *const *L, const int64_t *ldl,
                                   void *const *S, const int64_t *lds,
                                   int32_t *const *labels, respca_info *info, void *stream);

/*
 * Tile-shape tuner of the batched solver: times respca_solve_batched on the
 * given batch for each candidate (sweep columns per work item, rows per
 * distance slice, workgroups per compute unit) and keeps the fastest in the
 * handle.  With cache_path non-NULL the result is looked up in / appended to
 * that text file (one "key jc slice_rows blocks_per_cu ms" line per tuned size
 * bucket) so later processes skip the search.  Outputs are overwritten by the
 * timing runs.  best_ms (host, nullable) receives the winning time.
 */
respca_status respca_autotune_batched(respca_handle h, const respca_params *params, int32_t batch,
                                      const int64_t *d, const int64_t *n,
                                      const void *const *X, const int64_t *ldx,
                                      void *const *L, const int64_t *ldl,
                                      void *const *S, const int64_t *lds,
                                      const char *cache_path, double *best_ms, void *stream);

/*
 * The batched solver's tile shape, set by hand or read back (host values).
 * Accepted values are the tuner's candidates: jc (sweep columns per work item)
 * in {4, 8, 16, 32}, slice_rows (rows per distance slice) in {512, 1024, 2048},
 * blocks_per_cu (persistent workgroups per compute unit) in {1, 2}; anything
 * else is RESPCA_ERR_INVALID and leaves the shape unchanged.  The defaults are
 * (8, 1024, 2).  Needs no device.
 */
respca_status respca_set_batched_tile(respca_handle h, int32_t jc, int32_t slice_rows,
                                      int32_t blocks_per_cu);
respca_status respca_get_batched_tile(respca_handle h, int32_t *jc, int32_t *slice_rows,
                                      int32_t *blocks_per_cu);

/*
 * Kernel timing.  While enabled, every launch of the kernels listed in
 * respca_kernel_id is bracketed by HIP events recorded on the stream it is
 * launched on, and the library accumulates, per kernel, the number of
 * launches, their summed event time and their summed algorithmic HBM bytes
 * (the bytes the method must move: every d x n array the kernel reads or
 * writes once, at the element size of the run).  Enabling (or disabling)
 * resets the counters.  Timing adds two event records per timed launch, and
 * each record can leave the device idle for a few microseconds, so a caller
 * timing a whole solve may time only the unit it reports.
 */
typedef enum {
    RESPCA_KERNEL_SWEEP = 0,      /* fused L/S/Theta sweep: reads X, S, Theta, L; writes L, S, Theta */
    RESPCA_KERNEL_MEANS = 1,      /* group partial sums: reads X, S, Theta (or one array)            */
    RESPCA_KERNEL_DISTANCE = 2,   /* centroid . column products: reads the d x n operand once       */
    RESPCA_KERNEL_SEEDING = 3,    /* k-means++ squared distances: reads X once                      */
    RESPCA_KERNEL_BATCHED = 4,    /* one persistent batched launch (graph replay); bytes = the
                                     method's passes of every instance: 1 (||X||) + c (seeding)
                                     + 1 + 2 per initial Lloyd pass + 11 per outer iteration
                                     + 2 per extra Lloyd pass, times d n 4                          */
    RESPCA_KERNEL_COLNORM = 5,    /* l2,1 S-step column norms: reads X, S, Theta                     */
    RESPCA_KERNEL_AFFINITY = 6,   /* spectral p-step: Gram matrix on FP64 MFMA + Gaussian affinity;
                                     bytes = the d x n operand + the n x n FP64 affinity written,
                                     flops = n (n + 1) d (the symmetric half of Y^T Y)             */
    RESPCA_KERNEL_EIGEN = 7,      /* spectral p-step: one block product A Y (reads the n x n
                                     normalised affinity; flops 2 n^2 k, k = min(n, c + 8))        */
    RESPCA_KERNEL_COUNT = 8
} respca_kernel_id;

/* enable: 0 turns timing off; otherwise bit k (1 << k) times the launches of
 * respca_kernel_id k, and RESPCA_PROFILE_ALL times every unit. */
#define RESPCA_PROFILE_ALL (-1)
respca_status respca_profile_enable(respca_handle h, int32_t enable);
/* launches, total_ms, bytes and flops are host outputs (any may be NULL).
 * flops counts the algorithmic floating-point operations (the distance
 * contraction's 2 c d n per pass; zero for the streaming kernels). */
respca_status respca_profile_query(respca_handle h, int32_t kernel, int64_t *launches,
                                   double *total_ms, double *bytes, double *flops);

/*
 * Streaming bandwidth probe (measurement support, not part of the method): a
 * kernel that reads `reads` arrays (1..4) and writes `writes` arrays (0..3) of
 * bytes_per_array bytes each (a positive multiple of 16), float4 loads and
 * stores (nontemporal ones when `nontemporal` is nonzero, the form the sweep and
 * the means passes use on arrays of 64 MiB and more), launched reps times on
 * `stream` between two events after one warm-up launch.  *gbps (host) receives
 * (reads + writes) * bytes_per_array / time per launch, *ms_per_launch the mean
 * launch time (either may be NULL).  The arrays live in the handle's workspace
 * (allocated on demand).  The l1 sweep's mix on the compact state is 3 reads and
 * 2 writes, the l2,1 sweep's 4 and 3, a copy's 1 and 1.
 */
respca_status respca_bandwidth_probe(respca_handle h, int32_t reads, int32_t writes,
                                     int32_t nontemporal, int64_t bytes_per_array, int32_t reps,
                                     double *gbps, double *ms_per_launch, void *stream);

/*
 * Learned warm start (an addition to the paper's method; all FP32, device
 * pointers unless marked host).  A per-column network with dims
 * [68, hidden, hidden, hidden, 65] (ReLU between layers; parameters one flat
 * vector, layer by layer W (out x in, row-major) then b) maps each column's
 * normalised sketch and instance features to the normalised sketch of its group
 * centroid (64 outputs) and a log threshold (1 output).
 */
/* Number of network parameters (host).  Needs no device. */
int64_t       respca_mlp_param_count(int32_t hidden);
/* Floats of the activation buffer a forward pass for `batch` rows needs; the
 * network output (batch x 65, row-major) is its last block. Needs no device. */
int64_t       respca_mlp_act_count(int32_t hidden, int32_t batch);
/* Column sketch Y (65 x n, leading dimension 65): rows 0..63 are R X_j with
 * R[k][i] = +-1/8 from bit k of the i-th splitmix64(seed) output, row 64 ||X_j||. */
respca_status respca_sketch(respca_handle h, int64_t d, int64_t n, const void *X, int64_t ldx,
                            uint64_t seed, void *Y, void *stream);
/* Network inputs F (n x 68, row-major) from a sketch Y of a d x n matrix with c groups:
 * y_j / (s sqrt(d) / 8), log(||X_j|| / (s sqrt(d))), log(d)/8, log(n)/8, c/50 with
 * s = ||X||_F / sqrt(d n). */
respca_status respca_features(respca_handle h, int64_t d, int64_t n, int32_t c, const void *Y,
                              void *F, void *stream);
/* Forward pass over `batch` rows x (batch x 68); acts receives the activations. */
respca_status respca_mlp_forward(respca_handle h, int32_t hidden, const void *params, int32_t batch,
                                 const void *x, void *acts, void *stream);
/* Gradient (flat, like params) of sum(dy * output) given a forward pass's acts. */
respca_status respca_mlp_backward(respca_handle h, int32_t hidden, const void *params,
                                  int32_t batch, const void *x, const void *acts, const void *dy,
                                  void *grad, void *stream);
/* Loss (1/B) sum_j [sum_{k<64} (y - t)^2 + w_last (y_64 - t_64)^2] (host *loss) and dy. */
respca_status respca_mlp_loss(respca_handle h, int32_t batch, const void *y, const void *t,
                              float w_last, void *dy, double *loss, void *stream);
/* One Adam step (Kingma & Ba 2015, bias-corrected; step counts from 1). */
respca_status respca_mlp_adam(respca_handle h, int64_t count, void *params, const void *grad,
                              void *m, void *v, float lr, float beta1, float beta2, float eps,
                              int32_t step, void *stream);
/* Warm start of one d x n FP32 problem with c groups: sketch -> features ->
 * network -> initial labels = K-means (seed kmeans_seed) of the predicted centroid
 * sketches, rho0 (host) = exp(mean predicted log threshold) / s.  If the network's
 * threshold is not a finite positive number *fallback (host) is set to 1 and
 * *rho0 to 1e-4 (the default); the labels are always valid. */
respca_status respca_warmstart(respca_handle h, int32_t hidden, const void *params, int64_t d,
                               int64_t n, int32_t c, const void *X, int64_t ldx,
                               uint64_t sketch_seed, uint64_t kmeans_seed, int32_t *init_labels,
                               double *rho0, int32_t *fallback, void *stream);

/* Warm start of a batch of instances (the learned initialisation above, Sec. 4
 * groups and Sec. 4.4 rho, for every instance with one network pass over all
 * their columns).  Instance i is d[i] x n[i] (FP32, device, leading dimension
 * ldx[i]) with c[i] groups.  Writes `embedding` (device FP32, caller-allocated,
 * 65 x sum(n) column-major with leading dimension 65): the columns of instance i
 * start at column sum_{i' < i} n[i'], rows 0..63 hold the predicted centroid
 * sketches, to be passed as init_embedding (64 rows, leading dimension 65), row
 * 64 the predicted log-thresholds.  rho0[i] and fallback[i] (host arrays) as for
 * respca_warmstart.  At most 1024 instances; synchronises `stream`. */
respca_status respca_warmstart_batched(respca_handle h, int32_t hidden, const void *params,
                                       int32_t batch, const int64_t *d, const int64_t *n,
                                       const int32_t *c, const void *const *X, const int64_t *ldx,
                                       uint64_t sketch_seed, void *embedding, double *rho0,
                                       int32_t *fallback, void *stream);

/* Phase breakdown of the last batched launch: ms[p] for the phases
 * pack, init, seed-distance, seed-draw, seed-gather, sort, means, centroids
 * (with their norms), sweep, distance, argmin, control (count <= 12 entries are
 * written; each is the wall time one workgroup spent in that phase including its
 * barrier wait), and *steps the number of state-machine steps.  Host outputs. */
respca_status respca_profile_batched_phases(respca_handle h, double *ms, int32_t count,
                                            int64_t *steps);

#ifdef __cplusplus
}
#endif
#endif
