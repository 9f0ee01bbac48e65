/*
 * respca_oracle.c -- plain, slow FP64 CPU oracle for RES-PCA (arXiv 1904.07497).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  Written for
 * readability against the paper, not for speed: one loop per formula, in the
 * order the paper states the steps, every sum in index order.
 */
#include "respca_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG --- */

uint64_t oracle_splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double oracle_uniform01(uint64_t *state)
{
    return (double)(oracle_splitmix64_next(state) >> 11) * 0x1.0p-53;
}

uint64_t oracle_splitmix64_at(uint64_t seed, uint64_t t)
{
    uint64_t state = seed + t * 0x9E3779B97F4A7C15ULL;
    return oracle_splitmix64_next(&state);
}

/* ------------------------------------------------------------ sketch --- */

void oracle_sketch(int64_t d, int64_t n, const double *X, uint64_t seed, double *Y)
{
    for (int64_t j = 0; j < n; ++j) {
        double *y = Y + j * 65;
        for (int k = 0; k < 65; ++k) y[k] = 0.0;
        for (int64_t i = 0; i < d; ++i) {
            uint64_t bits = oracle_splitmix64_at(seed, (uint64_t)i);
            double x = X[j * d + i];
            for (int k = 0; k < 64; ++k) y[k] += ((bits >> k) & 1ULL) ? -0.125 * x : 0.125 * x;
            y[64] += x * x;
        }
        y[64] = sqrt(y[64]);
    }
}

/* ------------------------------------------------------------ helpers --- */

static double sq_dist(int64_t d, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < d; ++i) {
        double t = a[i] - b[i];
        s += t * t;
    }
    return s;
}

/* ------------------------------------------------------- group means --- */

void oracle_group_means(int64_t d, int64_t n, int32_t c, const double *Y,
                        const int32_t *labels, double *mean, int64_t *counts)
{
    double *sum = (double *)calloc((size_t)d * (size_t)c, sizeof(double));
    for (int32_t k = 0; k < c; ++k) counts[k] = 0;
    for (int64_t j = 0; j < n; ++j) {
        int32_t k = labels[j];
        counts[k] += 1;
        for (int64_t i = 0; i < d; ++i) sum[k * d + i] += Y[j * d + i];
    }
    for (int32_t k = 0; k < c; ++k) {
        if (counts[k] == 0) continue;
        for (int64_t i = 0; i < d; ++i) mean[k * d + i] = sum[k * d + i] / (double)counts[k];
    }
    free(sum);
}

/* ------------------------------------------------------------ L-step --- */

void oracle_l_step(int64_t d, int64_t n, int32_t c, double lambda, double rho,
                   const double *X, const double *S, const double *Theta,
                   const int32_t *labels, double *L, double *C)
{
    size_t dn = (size_t)d * (size_t)n;
    double *D = (double *)malloc(dn * sizeof(double));
    int64_t *counts = (int64_t *)malloc((size_t)c * sizeof(int64_t));

    /* D = X - S + Theta / rho  (the matrix the L-subproblem pulls L toward) */
    for (size_t e = 0; e < dn; ++e) D[e] = X[e] - S[e] + Theta[e] / rho;

    /* group means of D; the closed form needs the group sums divided by n_k */
    oracle_group_means(d, n, c, D, labels, C, counts);

    /* rho (2 lambda M_k + rho I)^{-1} = alpha I + (1 - alpha)/n_k 11^T with
     * alpha = rho/(2 lambda + rho) and 1 - alpha = 2 lambda/(2 lambda + rho):
     * each column keeps alpha of itself plus (1 - alpha) of its group mean. */
    double alpha = rho / (2.0 * lambda + rho);
    double beta = (2.0 * lambda) / (2.0 * lambda + rho);
    for (int64_t j = 0; j < n; ++j) {
        int32_t k = labels[j];
        for (int64_t i = 0; i < d; ++i)
            L[j * d + i] = alpha * D[j * d + i] + beta * C[k * d + i];
    }
    free(counts);
    free(D);
}

/* ------------------------------------------------------------ p-step --- */

void oracle_assign(int64_t d, int64_t n, int32_t c, const double *Y,
                   const double *C, int32_t *labels)
{
    for (int64_t j = 0; j < n; ++j) {
        int32_t best = 0;
        double bestd = sq_dist(d, Y + j * d, C);
        for (int32_t k = 1; k < c; ++k) {
            double dk = sq_dist(d, Y + j * d, C + (int64_t)k * d);
            if (dk < bestd) { bestd = dk; best = k; }
        }
        labels[j] = best;
    }
}

int32_t oracle_lloyd(int64_t d, int64_t n, int32_t c, const double *Y,
                     double *C, int32_t *labels, int32_t max_lloyd)
{
    int32_t *next = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *counts = (int64_t *)malloc((size_t)c * sizeof(int64_t));
    int32_t steps = 0;
    while (steps < max_lloyd) {
        oracle_assign(d, n, c, Y, C, next);
        ++steps;
        int changed = 0;
        for (int64_t j = 0; j < n; ++j) if (next[j] != labels[j]) { changed = 1; break; }
        if (!changed) break;
        memcpy(labels, next, (size_t)n * sizeof(int32_t));
        oracle_group_means(d, n, c, Y, labels, C, counts);
    }
    free(counts);
    free(next);
    return steps;
}

void oracle_kmeanspp(int64_t d, int64_t n, int32_t c, const double *Y,
                     uint64_t seed, int64_t *seeds)
{
    uint64_t state = seed;
    double *d2 = (double *)malloc((size_t)n * sizeof(double));
    char *chosen = (char *)calloc((size_t)n, 1);

    double u = oracle_uniform01(&state);
    int64_t s = (int64_t)floor(u * (double)n);
    if (s >= n) s = n - 1;
    seeds[0] = s;
    chosen[s] = 1;
    for (int64_t j = 0; j < n; ++j) d2[j] = sq_dist(d, Y + j * d, Y + s * d);

    for (int32_t m = 1; m < c; ++m) {
        double total = 0.0;
        for (int64_t j = 0; j < n; ++j) total += d2[j];
        u = oracle_uniform01(&state);
        s = -1;
        if (total > 0.0) {
            double target = u * total;
            double run = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                run += d2[j];
                if (run > target) { s = j; break; }
            }
            if (s < 0)
                for (int64_t j = n - 1; j >= 0; --j) if (d2[j] > 0.0) { s = j; break; }
        } else {
            for (int64_t j = 0; j < n; ++j) if (!chosen[j]) { s = j; break; }
        }
        if (s < 0) s = 0; /* unreachable: c <= n leaves an unchosen index */
        seeds[m] = s;
        chosen[s] = 1;
        for (int64_t j = 0; j < n; ++j) {
            double t = sq_dist(d, Y + j * d, Y + s * d);
            if (t < d2[j]) d2[j] = t;
        }
    }
    free(chosen);
    free(d2);
}

int32_t oracle_kmeans(int64_t d, int64_t n, int32_t c, const double *Y,
                      uint64_t seed, int32_t max_lloyd, int32_t *labels, double *C)
{
    int64_t *seeds = (int64_t *)malloc((size_t)c * sizeof(int64_t));
    int64_t *counts = (int64_t *)malloc((size_t)c * sizeof(int64_t));
    oracle_kmeanspp(d, n, c, Y, seed, seeds);
    for (int32_t k = 0; k < c; ++k) memcpy(C + (int64_t)k * d, Y + seeds[k] * d, (size_t)d * sizeof(double));
    oracle_assign(d, n, c, Y, C, labels);
    oracle_group_means(d, n, c, Y, labels, C, counts);
    int32_t steps = oracle_lloyd(d, n, c, Y, C, labels, max_lloyd);
    free(counts);
    free(seeds);
    return steps;
}

/* ------------------------------------------------------- S and Theta --- */

void oracle_s_step(int64_t d, int64_t n, double rho, const double *X,
                   const double *L, const double *Theta, double *S)
{
    size_t dn = (size_t)d * (size_t)n;
    double thr = 1.0 / rho;
    for (size_t e = 0; e < dn; ++e) {
        double b = X[e] - L[e] + Theta[e] / rho;
        double mag = fabs(b) - thr;
        if (mag < 0.0) mag = 0.0;
        S[e] = (b > 0.0) ? mag : ((b < 0.0) ? -mag : 0.0);
    }
}

void oracle_s_step_l21(int64_t d, int64_t n, double rho, const double *X,
                       const double *L, const double *Theta, double *S)
{
    for (int64_t j = 0; j < n; ++j) {
        const double *x = X + j * d, *l = L + j * d, *t = Theta + j * d;
        double *s = S + j * d;
        double nb2 = 0.0;
        for (int64_t i = 0; i < d; ++i) {
            double b = x[i] - l[i] + t[i] / rho;
            nb2 += b * b;
        }
        double nb = sqrt(nb2);
        double f = (rho * nb > 1.0) ? 1.0 - 1.0 / (rho * nb) : 0.0;
        for (int64_t i = 0; i < d; ++i) s[i] = f * (x[i] - l[i] + t[i] / rho);
    }
}

/* Sec. 5.3 (anomaly detection): the l2 norm of each column of S, the score by
   which the outlying samples are read off the recovered sparse part. */
void oracle_column_norms(int64_t d, int64_t n, const double *S, double *out)
{
    for (int64_t j = 0; j < n; ++j) {
        const double *s = S + j * d;
        double q = 0.0;
        for (int64_t i = 0; i < d; ++i) q += s[i] * s[i];
        out[j] = sqrt(q);
    }
}

void oracle_theta_step(int64_t d, int64_t n, double rho, const double *X,
                       const double *L, const double *S, double *Theta)
{
    size_t dn = (size_t)d * (size_t)n;
    for (size_t e = 0; e < dn; ++e) Theta[e] = Theta[e] + rho * (X[e] - L[e] - S[e]);
}

/* ------------------------------------------------------ one iteration --- */

int32_t oracle_step(const oracle_params *p, int64_t d, int64_t n, const double *X,
                    double *L, double *S, double *Theta, int32_t *labels,
                    double *C, double *rho, double norms[3])
{
    size_t dn = (size_t)d * (size_t)n;
    double *Lnew = (double *)malloc(dn * sizeof(double));
    double *Snew = (double *)malloc(dn * sizeof(double));
    double r = *rho;

    /* Sec. 4.1: L-step (C receives the group means of D) */
    oracle_l_step(d, n, p->c, p->lambda, r, X, S, Theta, labels, Lnew, C);
    /* Sec. 4.2: p-step = K-means of the columns of L, from the current groups */
    int32_t steps = oracle_lloyd(d, n, p->c, Lnew, C, labels, p->max_lloyd);
    /* Sec. 4.3: S-step (or its l2,1 form) */
    if (p->sparse_norm == 1) oracle_s_step_l21(d, n, r, X, Lnew, Theta, Snew);
    else oracle_s_step(d, n, r, X, Lnew, Theta, Snew);
    /* Sec. 4.4: multiplier and penalty */
    oracle_theta_step(d, n, r, X, Lnew, Snew, Theta);

    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
    for (size_t e = 0; e < dn; ++e) {
        double a = X[e] - Lnew[e] - Snew[e];
        double b = Lnew[e] - L[e];
        double s = Snew[e] - S[e];
        r0 += a * a;
        r1 += b * b;
        r2 += s * s;
    }
    norms[0] = sqrt(r0);
    norms[1] = sqrt(r1);
    norms[2] = sqrt(r2);

    memcpy(L, Lnew, dn * sizeof(double));
    memcpy(S, Snew, dn * sizeof(double));
    double next = p->kappa * r;
    *rho = (next < p->rho_max) ? next : p->rho_max;
    free(Snew);
    free(Lnew);
    return steps;
}

void oracle_step_columns(const oracle_params *p, int64_t d, int64_t n, const double *X,
                         const double *S, const double *Theta, const int32_t *labels,
                         const double *C, double rho, int64_t nsel, const int64_t *sel,
                         double *L_out, double *S_out, double *Theta_out, int32_t *labels_out,
                         double *mu_out)
{
    size_t dn = (size_t)d * (size_t)n;
    int32_t c = p->c;
    double *D = (double *)malloc(dn * sizeof(double));
    double *mu = (double *)malloc((size_t)d * (size_t)c * sizeof(double));
    int64_t *counts = (int64_t *)malloc((size_t)c * sizeof(int64_t));
    for (size_t e = 0; e < dn; ++e) D[e] = X[e] - S[e] + Theta[e] / rho;
    memcpy(mu, C, (size_t)d * (size_t)c * sizeof(double));
    oracle_group_means(d, n, c, D, labels, mu, counts);   /* empty groups keep C */

    double alpha = rho / (2.0 * p->lambda + rho);
    double beta = (2.0 * p->lambda) / (2.0 * p->lambda + rho);
    for (int64_t q = 0; q < nsel; ++q) {
        int64_t j = sel[q];
        int32_t k = labels[j];
        double *Lq = L_out + q * d;
        for (int64_t i = 0; i < d; ++i) Lq[i] = alpha * D[j * d + i] + beta * mu[k * d + i];
        oracle_assign(d, 1, c, Lq, mu, labels_out + q);
        if (p->sparse_norm == 1) oracle_s_step_l21(d, 1, rho, X + j * d, Lq, Theta + j * d, S_out + q * d);
        else oracle_s_step(d, 1, rho, X + j * d, Lq, Theta + j * d, S_out + q * d);
        memcpy(Theta_out + q * d, Theta + j * d, (size_t)d * sizeof(double));
        oracle_theta_step(d, 1, rho, X + j * d, Lq, S_out + q * d, Theta_out + q * d);
    }
    if (mu_out) memcpy(mu_out, mu, (size_t)d * (size_t)c * sizeof(double));
    free(counts);
    free(mu);
    free(D);
}

/* --------------------------------------------------------- whole solve --- */

static int params_valid(const oracle_params *p, int64_t d, int64_t n)
{
    if (d < 1 || n < 1) return 0;
    if (p->c < 1 || (int64_t)p->c > n) return 0;
    if (!(p->lambda >= 0.0) || !isfinite(2.0 * p->lambda)) return 0;
    if (!(p->rho0 > 0.0) || !isfinite(p->rho0)) return 0;
    if (!(p->kappa > 1.0) || !isfinite(p->kappa)) return 0;
    if (!(p->rho_max >= p->rho0)) return 0;
    if (!(p->tol >= 0.0)) return 0;
    if (p->sparse_norm != 0 && p->sparse_norm != 1) return 0;
    if (p->max_iter < 1 || p->max_lloyd < 1) return 0;
    return 1;
}

int32_t oracle_solve(const oracle_params *p, int64_t d, int64_t n, const double *X,
                     double *L, double *S, int32_t *labels, double *C,
                     const int32_t *init_labels, oracle_info *info, double *history)
{
    memset(info, 0, sizeof(*info));
    if (!params_valid(p, d, n)) { info->status = ORACLE_ERR_INVALID; return info->status; }
    if (init_labels)
        for (int64_t j = 0; j < n; ++j)
            if (init_labels[j] < 0 || init_labels[j] >= p->c) {
                info->status = ORACLE_ERR_INVALID;
                return info->status;
            }

    size_t dn = (size_t)d * (size_t)n;
    double nx2 = 0.0;
    for (size_t e = 0; e < dn; ++e) nx2 += X[e] * X[e];
    if (!isfinite(nx2)) { info->status = ORACLE_ERR_NONFINITE; return info->status; }

    memset(L, 0, dn * sizeof(double));
    memset(S, 0, dn * sizeof(double));
    if (nx2 == 0.0) {
        memset(labels, 0, (size_t)n * sizeof(int32_t));
        memset(C, 0, (size_t)d * (size_t)p->c * sizeof(double));
        info->status = ORACLE_OK;
        return ORACLE_OK;
    }
    double nX = sqrt(nx2);

    /* initial groups: K-means of the columns of X (or the caller's labels) */
    if (init_labels) {
        int64_t *counts = (int64_t *)malloc((size_t)p->c * sizeof(int64_t));
        memcpy(labels, init_labels, (size_t)n * sizeof(int32_t));
        memset(C, 0, (size_t)d * (size_t)p->c * sizeof(double));
        oracle_group_means(d, n, p->c, X, labels, C, counts);
        free(counts);
    } else {
        info->init_lloyd = oracle_kmeans(d, n, p->c, X, p->seed, p->max_lloyd, labels, C);
    }

    double *Theta = (double *)calloc(dn, sizeof(double));
    double rho = p->rho0;
    info->status = ORACLE_NOT_CONVERGED;
    for (int32_t t = 1; t <= p->max_iter; ++t) {
        double norms[3];
        double rho_t = rho;
        info->lloyd_steps += oracle_step(p, d, n, X, L, S, Theta, labels, C, &rho, norms);
        info->iters = t;
        info->rho_final = rho_t;
        info->primal = norms[0] / nX;
        info->dL = norms[1] / nX;
        info->dS = norms[2] / nX;
        if (history) {
            history[3 * (t - 1) + 0] = info->primal;
            history[3 * (t - 1) + 1] = info->dL;
            history[3 * (t - 1) + 2] = info->dS;
        }
        double crit = info->primal;
        if (info->dL > crit) crit = info->dL;
        if (info->dS > crit) crit = info->dS;
        if (crit <= p->tol) { info->status = ORACLE_OK; break; }
    }
    free(Theta);
    return info->status;
}
