/*
 * respca_oracle.h -- plain, slow FP64 CPU oracle for RES-PCA
 * (Peng et al., "RES-PCA: A Scalable Approach to Recovering Low-rank
 * Matrices", arXiv 1904.07497).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists so that the GPU library can be
 * checked against an obviously-correct implementation.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load or call it;
 * the GPU library never links, includes or calls anything in this directory,
 * and this directory includes nothing from the GPU library.
 *
 * Conventions
 *   - Every matrix is d x n, column-major, contiguous (leading dimension d):
 *     element (i, j) is M[j*d + i].  Column j is sample j (Sec. 3: the columns
 *     of X are the data points).
 *   - labels[j] in [0, c) is the group of column j; it is the one-hot
 *     indicator p_1..p_c of the model (eq. eq_obj) stored as an index.
 *   - Group sizes n_k are the number of ones in p_k (the paper writes
 *     ||p_k||_2 for it; only the count makes the matrices of the L-step
 *     well defined, see the readings in the design notes).
 *   - All arithmetic is IEEE double, no fast-math, loops in index order.
 */
#ifndef RESPCA_ORACLE_H
#define RESPCA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double   lambda;     /* weight of the group-variance (trace) term of eq_obj            */
    int32_t  c;          /* number of groups                                               */
    double   tol;        /* stopping tolerance of the relative criterion (Sec. 5)          */
    int32_t  max_iter;   /* outer ALM iterations cap (Sec. 5: 500)                          */
    double   rho0;       /* initial penalty (Sec. 5.1: 1e-4)                                */
    double   kappa;      /* penalty growth factor > 1 (Sec. 4.4; Sec. 5.1: 1.5)             */
    double   rho_max;    /* cap on rho (not in the paper)                                   */
    int32_t  max_lloyd;  /* cap on Lloyd assignment passes per K-means call                 */
    uint64_t seed;       /* k-means++ seeding stream                                        */
    int32_t  sparse_norm;/* penalty on S: 0 the l1 norm of eq_obj (Sec. 3), 1 the column-wise
                            l2,1 norm named as the alternative after eq_obj (Sec. 3); the
                            norm is defined with eq_rpca_l21 (Sec. 2); other values invalid */
} oracle_params;

typedef struct {
    int32_t iters;        /* outer iterations run                                         */
    int32_t lloyd_steps;  /* assignment passes summed over the outer iterations           */
    int32_t init_lloyd;   /* assignment passes of the initial K-means on X                */
    int32_t status;       /* 0 converged, 1 not converged, <0 error                       */
    double  primal;       /* ||X-L-S||_F / ||X||_F at the last iteration                  */
    double  dL;           /* ||L_t - L_{t-1}||_F / ||X||_F                                */
    double  dS;           /* ||S_t - S_{t-1}||_F / ||X||_F                                */
    double  rho_final;    /* rho used by the last iteration                               */
} oracle_info;

#define ORACLE_OK             0
#define ORACLE_NOT_CONVERGED  1
#define ORACLE_ERR_INVALID   -1
#define ORACLE_ERR_NONFINITE -2

/* splitmix64 (Steele, Lea & Flood, OOPSLA 2014): advance the state by the
 * golden-gamma constant and return the mixed 64-bit output. */
uint64_t oracle_splitmix64_next(uint64_t *state);
/* Uniform double in [0, 1): the top 53 bits of the next output times 2^-53. */
double oracle_uniform01(uint64_t *state);
/* Counter-based access: the (t+1)-th output of splitmix64 started from `seed`. */
uint64_t oracle_splitmix64_at(uint64_t seed, uint64_t t);

/* Column sketch used by the learned warm start (not part of the paper's method):
 * Y (65 x n, leading dimension 65): rows 0..63 are R X_j with R[k][i] = +1/8 if
 * bit k of oracle_splitmix64_at(seed, i) is 0 and -1/8 otherwise (a Rademacher
 * random projection), row 64 is ||X_j||_2. */
void oracle_sketch(int64_t d, int64_t n, const double *X, uint64_t seed, double *Y);

/* Group means: for every k with n_k > 0, mean[:, k] = (1/n_k) sum_{labels[j]=k} Y[:, j].
 * Columns of empty groups are left untouched.  counts[k] = n_k. */
void oracle_group_means(int64_t d, int64_t n, int32_t c, const double *Y,
                        const int32_t *labels, double *mean, int64_t *counts);

/* L-step, Sec. 4.1 (closed form after the Sherman-Morrison-Woodbury inverse):
 * D = X - S + Theta/rho; for column j of group k,
 *   L_j = rho/(2 lambda + rho) D_j + 2 lambda/(n_k (2 lambda + rho)) sum_{j' in k} D_j'.
 * C[:, k] is overwritten with the group mean of D for every non-empty group. */
void oracle_l_step(int64_t d, int64_t n, int32_t c, double lambda, double rho,
                   const double *X, const double *S, const double *Theta,
                   const int32_t *labels, double *L, double *C);

/* Nearest-centroid assignment: labels[j] = argmin_k sum_i (Y_ij - C_ik)^2,
 * computed in the difference form; ties go to the lowest k. */
void oracle_assign(int64_t d, int64_t n, int32_t c, const double *Y,
                   const double *C, int32_t *labels);

/* Lloyd iterations for K-means (the p-step of Sec. 4.2) started from
 * (labels, C): assign; stop if no label changed; otherwise replace labels and
 * set C to the group means of Y (empty groups keep their centroid); at most
 * max_lloyd assignment passes.  Returns the number of assignment passes. */
int32_t oracle_lloyd(int64_t d, int64_t n, int32_t c, const double *Y,
                     double *C, int32_t *labels, int32_t max_lloyd);

/* k-means++ seeding (Arthur & Vassilvitskii 2007) driven by splitmix64(seed).
 * seeds[0] = floor(u n); each next seed is drawn with probability proportional
 * to the squared distance to the nearest chosen seed, by inverse CDF over the
 * running sum in index order (first j whose running sum exceeds u * total).
 * When every squared distance is zero the lowest index not yet chosen is taken;
 * when rounding leaves no running sum above u * total the last index with a
 * non-zero squared distance is taken.  One draw of u per seed, always. */
void oracle_kmeanspp(int64_t d, int64_t n, int32_t c, const double *Y,
                     uint64_t seed, int64_t *seeds);

/* K-means of the columns of Y: k-means++ seeds, nearest-seed assignment,
 * centroids = group means (an empty group keeps its seed), then oracle_lloyd.
 * Returns the number of Lloyd assignment passes. */
int32_t oracle_kmeans(int64_t d, int64_t n, int32_t c, const double *Y,
                      uint64_t seed, int32_t max_lloyd, int32_t *labels, double *C);

/* S-step, Sec. 4.3: B = X - L + Theta/rho, S = sign(B) max(|B| - 1/rho, 0). */
void oracle_s_step(int64_t d, int64_t n, double rho, const double *X,
                   const double *L, const double *Theta, double *S);
/* S-step with the l2,1 norm: column j of S is B_j max(0, 1 - 1/(rho ||B_j||)),
 * B = X - L + Theta/rho (the proximal map of (1/rho)||.||_2 per column). */
void oracle_s_step_l21(int64_t d, int64_t n, double rho, const double *X,
                       const double *L, const double *Theta, double *S);

/* Multiplier update, Sec. 4.4: Theta <- Theta + rho (X - L - S). */
void oracle_theta_step(int64_t d, int64_t n, double rho, const double *X,
                       const double *L, const double *S, double *Theta);

/* One outer ALM iteration (Sec. 4 in section order: L, p, S, Theta/rho).
 * On entry L holds L_{t-1} (zeros before the first iteration), S and Theta the
 * previous iterate, labels/C the current groups and centroids, *rho = rho_t.
 * On exit L, S, Theta, labels, C hold iterate t, *rho = min(kappa rho_t, rho_max)
 * and norms[0..2] = ||X - L_t - S_t||_F, ||L_t - L_{t-1}||_F, ||S_t - S_{t-1}||_F.
 * Returns the number of Lloyd assignment passes. */
int32_t oracle_step(const oracle_params *p, int64_t d, int64_t n, const double *X,
                    double *L, double *S, double *Theta, int32_t *labels,
                    double *C, double *rho, double norms[3]);

/* One outer iteration restricted to selected columns, with a single assignment
 * pass (max_lloyd = 1): the group means of D are taken over ALL n columns, then
 * for each selected column sel[q] the outputs L, S, Theta (d values each, stored
 * as column q of d x nsel arrays) and its new label are computed from them.
 * C (d x c, in) supplies the centroid of groups that are empty; mu_out
 * (d x c, nullable) receives the centroids the assignment used.  Used to check
 * large runs column by column. */
void oracle_step_columns(const oracle_params *p, int64_t d, int64_t n, const double *X,
                         const double *S, const double *Theta, const int32_t *labels,
                         const double *C, double rho, int64_t nsel, const int64_t *sel,
                         double *L_out, double *S_out, double *Theta_out, int32_t *labels_out,
                         double *mu_out);

/* Whole solve.  init_labels (nullable) replaces the k-means++ initialisation;
 * the centroids then start as group means of X (zero for empty groups).
 * history (nullable) receives 3 doubles per iteration (the relative criterion
 * terms).  labels and C (d x c) are outputs.  Returns the status. */
int32_t oracle_solve(const oracle_params *p, int64_t d, int64_t n, const double *X,
                     double *L, double *S, int32_t *labels, double *C,
                     const int32_t *init_labels, oracle_info *info, double *history);

#ifdef __cplusplus
}
#endif
#endif
