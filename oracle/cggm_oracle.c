/*
 * cggm_oracle.c -- plain FP64 CPU reference of alternating Newton coordinate
 * descent (ANCD) for the l1-regularized CGGM of McCarter & Kim (AISTATS 2016).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * measured against: it is deliberately slow and written to be read against
 * the paper -- dense row-major matrices, textbook loops, sequential
 * Gauss-Seidel coordinate descent in lexicographic order, its own Cholesky.
 * OpenMP pragmas only split the outer loops of plain dense products.  It
 * shares no code with the GPU library and is never linked into it.
 *
 * Where the paper is silent or its appendix is garbled, this file follows the
 * readings below (derived from Eq. (1), (3) and (4)):
 *   - Lambda CD curvature (appendix, Lambda update): for i != j the pair
 *     (i,j),(j,i) moves together and the exact curvature of the quadratic model
 *     along that direction, halved, is
 *       a = S_ij^2 + S_ii S_jj + S_ii P_jj + S_jj P_ii + 2 S_ij P_ij
 *     (S = Sigma, P = Psi); the printed formula is not symmetric in i,j.
 *     For i == j: a = S_ii^2 + 2 S_ii P_ii.
 *   - Theta CD curvature (appendix, Theta update): a = 2 Sigma_jj Sxx_ii, the
 *     second derivative of g along Theta_ij (the printed value is half of it).
 *   - Psi = Sigma Theta^T Sxx Theta Sigma exactly as defined after Eq. (4).
 *   - Both triangles and the diagonal of Lambda are penalized (elementwise l1).
 *   - Line search: Armijo on f with beta = 0.5, sigma = 1e-3 supplied by the
 *     caller, positive definiteness tested by Cholesky success; the test allows
 *     1e-14 max(1, |f|) for the rounding error of f itself.
 *   - Screening uses strict '>' against lambda and an exact-zero test.
 */
#define _DEFAULT_SOURCE   /* posix_memalign, madvise */
#include "cggm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>

#define IDX(i, j, ld) ((size_t)(i) * (size_t)(ld) + (size_t)(j))

/* Relative size of the rounding error of an FP64 objective evaluation. */
#define ARMIJO_ROUNDING 1e-14

/* Products below this many multiply-adds run on one thread. */
#define OMP_MIN_WORK 4000000LL

/* Zeroed array.  Large ones are backed by 2 MiB pages where the kernel
 * allows it: the coordinate sweeps walk columns of row-major matrices, and
 * with 4 KiB pages nearly every such access misses the TLB. */
static double *zalloc(size_t count) {
    const size_t bytes = (count ? count : 1) * sizeof(double), huge = (size_t)2 << 20;
    if (bytes < 2 * huge) {
        double *p = (double *)calloc(count ? count : 1, sizeof(double));
        if (!p) abort();
        return p;
    }
    void *p = NULL;
    const size_t rounded = (bytes + huge - 1) / huge * huge;
    if (posix_memalign(&p, huge, rounded) != 0) abort();
    (void)madvise(p, rounded, MADV_HUGEPAGE);
    memset(p, 0, bytes);
    return (double *)p;
}

/* C = A B (A m x k, B k x nc), skipping zero entries of A. */
static void matmul(int64_t m, int64_t k, int64_t nc, const double *A, const double *B,
                   double *C) {
#pragma omp parallel for schedule(static) if (m * k * nc > OMP_MIN_WORK)
    for (int64_t i = 0; i < m; ++i) {
        double *c = C + IDX(i, 0, nc);
        for (int64_t j = 0; j < nc; ++j) c[j] = 0.0;
        for (int64_t l = 0; l < k; ++l) {
            double a = A[IDX(i, l, k)];
            if (a == 0.0) continue;
            const double *b = B + IDX(l, 0, nc);
            for (int64_t j = 0; j < nc; ++j) c[j] += a * b[j];
        }
    }
}

/* C = A^T B (A k x m, B k x nc), skipping zero entries of A. */
static void matmul_tn(int64_t m, int64_t k, int64_t nc, const double *A, const double *B,
                      double *C) {
#pragma omp parallel for schedule(static) if (m * k * nc > OMP_MIN_WORK)
    for (int64_t i = 0; i < m; ++i) {
        double *c = C + IDX(i, 0, nc);
        for (int64_t j = 0; j < nc; ++j) c[j] = 0.0;
        for (int64_t l = 0; l < k; ++l) {
            double a = A[IDX(l, i, m)];
            if (a == 0.0) continue;
            const double *b = B + IDX(l, 0, nc);
            for (int64_t j = 0; j < nc; ++j) c[j] += a * b[j];
        }
    }
}

static double soft_threshold(double w, double r) {
    /* S_r(w) = sign(w) max(|w| - r, 0)  (appendix) */
    double m = fabs(w) - r;
    if (m <= 0.0) return 0.0;
    return w > 0.0 ? m : -m;
}

static double l1_norm(size_t count, const double *A) {
    double s = 0.0;
    for (size_t i = 0; i < count; ++i) s += fabs(A[i]);
    return s;
}

void orc_stats(int64_t n, int64_t p, int64_t q, const double *X, const double *Y,
               double *Sxx, double *Sxy, double *Syy) {
    /* Sxx = X^T X / n, Sxy = X^T Y / n, Syy = Y^T Y / n (Sec. 2.1, no centering) */
    matmul_tn(p, n, p, X, X, Sxx);
    matmul_tn(p, n, q, X, Y, Sxy);
    matmul_tn(q, n, q, Y, Y, Syy);
    double s = 1.0 / (double)n;
    for (size_t i = 0; i < (size_t)(p * p); ++i) Sxx[i] *= s;
    for (size_t i = 0; i < (size_t)(p * q); ++i) Sxy[i] *= s;
    for (size_t i = 0; i < (size_t)(q * q); ++i) Syy[i] *= s;
}

int orc_cholesky(int64_t q, const double *A, double *L) {
    /* Cholesky-Banachiewicz: L_jj = sqrt(A_jj - sum_k L_jk^2),
     * L_ij = (A_ij - sum_k L_ik L_jk) / L_jj for i > j. */
    memset(L, 0, sizeof(double) * (size_t)(q * q));
    for (int64_t j = 0; j < q; ++j) {
        double d = A[IDX(j, j, q)];
        for (int64_t k = 0; k < j; ++k) d -= L[IDX(j, k, q)] * L[IDX(j, k, q)];
        if (!(d > 0.0)) return ORC_NOTPD;
        double ljj = sqrt(d);
        L[IDX(j, j, q)] = ljj;
#pragma omp parallel for schedule(static) if ((q - j) * j > OMP_MIN_WORK / 16)
        for (int64_t i = j + 1; i < q; ++i) {
            double s = A[IDX(i, j, q)];
            for (int64_t k = 0; k < j; ++k) s -= L[IDX(i, k, q)] * L[IDX(j, k, q)];
            L[IDX(i, j, q)] = s / ljj;
        }
    }
    return ORC_OK;
}

void orc_inverse_from_cholesky(int64_t q, const double *L, double *Sigma) {
    /* W = L^{-1} by forward substitution on the identity, then Sigma = W^T W. */
    double *W = zalloc((size_t)(q * q));
#pragma omp parallel for schedule(dynamic, 8) if (q * q * q > OMP_MIN_WORK)
    for (int64_t c = 0; c < q; ++c) {          /* column c of W solves L w = e_c */
        for (int64_t i = c; i < q; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int64_t k = c; k < i; ++k) s -= L[IDX(i, k, q)] * W[IDX(k, c, q)];
            W[IDX(i, c, q)] = s / L[IDX(i, i, q)];
        }
    }
    matmul_tn(q, q, q, W, W, Sigma);
    free(W);
}

static double logdet_from_cholesky(int64_t q, const double *L) {
    double s = 0.0;
    for (int64_t i = 0; i < q; ++i) s += log(L[IDX(i, i, q)]);
    return 2.0 * s;
}

/* f from precomputed pieces: M = Theta^T Sxx Theta (q x q), Sigma, log det. */
static double objective_from_parts(int64_t p, int64_t q, const double *Sxy,
                                   const double *Syy, const double *Lambda,
                                   const double *Theta, const double *Sigma,
                                   const double *M, double logdet, double lamL,
                                   double lamT) {
    double tr_syy = 0.0, tr_sxy = 0.0, tr_sm = 0.0;
    for (int64_t i = 0; i < q; ++i)
        for (int64_t j = 0; j < q; ++j) {
            tr_syy += Syy[IDX(i, j, q)] * Lambda[IDX(j, i, q)];   /* tr(Syy Lambda) */
            tr_sm += Sigma[IDX(i, j, q)] * M[IDX(j, i, q)];       /* tr(Sigma M)    */
        }
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < q; ++j) tr_sxy += Sxy[IDX(i, j, q)] * Theta[IDX(i, j, q)];
    return -logdet + tr_syy + 2.0 * tr_sxy + tr_sm +
           lamL * l1_norm((size_t)(q * q), Lambda) + lamT * l1_norm((size_t)(p * q), Theta);
}

/* M = Theta^T Sxx Theta */
static void theta_sxx_theta(int64_t p, int64_t q, const double *Sxx, const double *Theta,
                            double *M) {
    double *T1 = zalloc((size_t)(p * q));
    matmul(p, p, q, Sxx, Theta, T1);          /* Sxx Theta */
    matmul_tn(q, p, q, Theta, T1, M);          /* Theta^T (Sxx Theta) */
    free(T1);
}

int orc_objective(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                  const double *Syy, const double *Lambda, const double *Theta,
                  double lamL, double lamT, double *f) {
    /* Eq. (1): f = -log|Lambda| + tr(Syy Lambda + 2 Sxy^T Theta
     *              + Lambda^{-1} Theta^T Sxx Theta) + lamL ||Lambda||_1 + lamT ||Theta||_1 */
    double *L = zalloc((size_t)(q * q));
    if (orc_cholesky(q, Lambda, L) != ORC_OK) {
        free(L);
        return ORC_NOTPD;
    }
    double *Sigma = zalloc((size_t)(q * q)), *M = zalloc((size_t)(q * q));
    orc_inverse_from_cholesky(q, L, Sigma);
    theta_sxx_theta(p, q, Sxx, Theta, M);
    *f = objective_from_parts(p, q, Sxy, Syy, Lambda, Theta, Sigma, M,
                              logdet_from_cholesky(q, L), lamL, lamT);
    free(L);
    free(Sigma);
    free(M);
    return ORC_OK;
}

/* Sigma, Psi, Gamma-based gradient; Sigma must already be Lambda^{-1}. */
static void gradient_given_sigma(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                                 const double *Syy, const double *Theta,
                                 const double *Sigma, double *GL, double *GT, double *Psi,
                                 double *M_out) {
    double *T1 = zalloc((size_t)(p * q)), *Gam = zalloc((size_t)(p * q));
    double *M = zalloc((size_t)(q * q)), *SM = zalloc((size_t)(q * q));
    matmul(p, p, q, Sxx, Theta, T1);           /* Sxx Theta                  */
    matmul(p, q, q, T1, Sigma, Gam);           /* Gamma = Sxx Theta Sigma    */
    matmul_tn(q, p, q, Theta, T1, M);          /* M = Theta^T Sxx Theta      */
    matmul(q, q, q, Sigma, M, SM);
    matmul(q, q, q, SM, Sigma, Psi);           /* Psi = Sigma M Sigma        */
    for (size_t i = 0; i < (size_t)(q * q); ++i) GL[i] = Syy[i] - Sigma[i] - Psi[i];
    for (size_t i = 0; i < (size_t)(p * q); ++i) GT[i] = 2.0 * Sxy[i] + 2.0 * Gam[i];
    if (M_out) memcpy(M_out, M, sizeof(double) * (size_t)(q * q));
    free(T1);
    free(Gam);
    free(M);
    free(SM);
}

int orc_gradient(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                 const double *Syy, const double *Lambda, const double *Theta,
                 double *GL, double *GT, double *Sigma_out, double *Psi_out) {
    double *L = zalloc((size_t)(q * q));
    if (orc_cholesky(q, Lambda, L) != ORC_OK) {
        free(L);
        return ORC_NOTPD;
    }
    double *Sigma = zalloc((size_t)(q * q)), *Psi = zalloc((size_t)(q * q));
    orc_inverse_from_cholesky(q, L, Sigma);
    gradient_given_sigma(p, q, Sxx, Sxy, Syy, Theta, Sigma, GL, GT, Psi, NULL);
    if (Sigma_out) memcpy(Sigma_out, Sigma, sizeof(double) * (size_t)(q * q));
    if (Psi_out) memcpy(Psi_out, Psi, sizeof(double) * (size_t)(q * q));
    free(L);
    free(Sigma);
    free(Psi);
    return ORC_OK;
}

void orc_active_sets(int64_t p, int64_t q, const double *GL, const double *GT,
                     const double *Lambda, const double *Theta, double lamL,
                     double lamT, uint8_t *actL, uint8_t *actT) {
    /* S = {|grad_ij| > lambda  or  param_ij != 0}  (Sec. 2.2) */
    for (int64_t i = 0; i < q; ++i)
        for (int64_t j = 0; j < q; ++j) {
            size_t k = IDX(i, j, q);
            actL[k] = (j >= i) && (fabs(GL[k]) > lamL || Lambda[k] != 0.0);
        }
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < q; ++j) {
            size_t k = IDX(i, j, q);
            actT[k] = fabs(GT[k]) > lamT || Theta[k] != 0.0;
        }
}

void orc_lambda_direction(int64_t q, const double *Sigma, const double *Psi,
                          const double *GL, const double *Lambda, const uint8_t *actL,
                          double lamL, int passes, double *D) {
    /* Coordinate descent on  gbar(D) + lamL ||Lambda + D||_1  (Eq. (6)), with the
     * quadratic model gbar(D) = tr(G D) + 1/2 tr(D Sigma D Sigma) + tr(D Sigma D Psi)
     * (Hessian Sigma (x) (Sigma + 2 Psi), Eq. (4)).  U = D Sigma is maintained. */
    double *U = zalloc((size_t)(q * q));
    memset(D, 0, sizeof(double) * (size_t)(q * q));
    for (int pass = 0; pass < passes; ++pass)
    for (int64_t i = 0; i < q; ++i) {
        for (int64_t j = i; j < q; ++j) {
            if (!actL[IDX(i, j, q)]) continue;
            const double *Si = Sigma + IDX(i, 0, q), *Sj = Sigma + IDX(j, 0, q);
            const double *Pi = Psi + IDX(i, 0, q), *Pj = Psi + IDX(j, 0, q);
            double sij = Si[j], sii = Si[i], sjj = Sj[j];
            double pij = Pi[j], pii = Pi[i], pjj = Pj[j];
            /* b = G_ij + (Sigma D Sigma)_ij + (Psi D Sigma)_ij + (Psi D Sigma)_ji */
            double sdsig = 0.0, pds_ij = 0.0, pds_ji = 0.0;
            for (int64_t k = 0; k < q; ++k) {
                sdsig += Si[k] * U[IDX(k, j, q)];
                pds_ij += Pi[k] * U[IDX(k, j, q)];
                pds_ji += Pj[k] * U[IDX(k, i, q)];
            }
            double b = GL[IDX(i, j, q)] + sdsig + pds_ij + pds_ji;
            double a = (i == j) ? sii * sii + 2.0 * sii * pii
                                : sij * sij + sii * sjj + sii * pjj + sjj * pii + 2.0 * sij * pij;
            if (!(a > 0.0)) continue;
            double c = Lambda[IDX(i, j, q)] + D[IDX(i, j, q)];
            /* minimizer of 1/2 a mu^2 + b mu + lamL |c + mu|:
             * mu = -c + S_{lamL/a}(c - b/a)  (appendix) */
            double mu = -c + soft_threshold(c - b / a, lamL / a);
            if (mu == 0.0) continue;
            D[IDX(i, j, q)] += mu;
            if (i != j) D[IDX(j, i, q)] += mu;
            /* U = D Sigma: row i gains mu Sigma_j., row j gains mu Sigma_i. */
            double *Ui = U + IDX(i, 0, q);
            for (int64_t k = 0; k < q; ++k) Ui[k] += mu * Sj[k];
            if (i != j) {
                double *Uj = U + IDX(j, 0, q);
                for (int64_t k = 0; k < q; ++k) Uj[k] += mu * Si[k];
            }
        }
    }
    free(U);
}

int orc_line_search(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                    const double *Syy, double *Lambda, const double *Theta,
                    const double *D, const double *GL, double lamL, double lamT,
                    double f0, double beta, double sigma, int max_ls,
                    double *alpha_out, double *f_out, int *trials_out) {
    /* Armijo rule: accept the first alpha in 1, beta, beta^2, ... for which
     * Lambda + alpha D is positive definite and
     * f(Lambda + alpha D, Theta) <= f0 + sigma alpha delta, with
     * delta = tr(G_Lambda D) + lamL (||Lambda + D||_1 - ||Lambda||_1). */
    size_t qq = (size_t)(q * q);
    double trGD = 0.0, l1diff = 0.0;
    for (size_t k = 0; k < qq; ++k) {
        trGD += GL[k] * D[k];
        l1diff += fabs(Lambda[k] + D[k]) - fabs(Lambda[k]);   /* entrywise: no cancellation */
    }
    double delta = trGD + lamL * l1diff;
    *alpha_out = 0.0;
    *f_out = f0;
    *trials_out = 0;
    if (!(delta < 0.0)) return ORC_OK;     /* no descent: Lambda already optimal given Theta */
    double *M = zalloc(qq), *Lt = zalloc(qq), *Lc = zalloc(qq), *Sg = zalloc(qq);
    theta_sxx_theta(p, q, Sxx, Theta, M);
    double alpha = 1.0;
    int accepted = 0;
    for (int t = 0; t < max_ls; ++t, alpha *= beta) {
        ++*trials_out;
        for (size_t k = 0; k < qq; ++k) Lt[k] = Lambda[k] + alpha * D[k];
        if (orc_cholesky(q, Lt, Lc) != ORC_OK) continue;
        orc_inverse_from_cholesky(q, Lc, Sg);
        double fa = objective_from_parts(p, q, Sxy, Syy, Lt, Theta, Sg, M,
                                         logdet_from_cholesky(q, Lc), lamL, lamT);
        /* the allowance covers the rounding error of evaluating f, so steps
         * whose true decrease is below it are not rejected as increases */
        if (fa <= f0 + sigma * alpha * delta + ARMIJO_ROUNDING * fmax(1.0, fabs(f0))) {
            memcpy(Lambda, Lt, sizeof(double) * qq);
            *alpha_out = alpha;
            *f_out = fa;
            accepted = 1;
            break;
        }
    }
    free(M);
    free(Lt);
    free(Lc);
    free(Sg);
    return accepted ? ORC_OK : ORC_MAXITER;
}

void orc_theta_sweep(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                     const double *Sigma, const uint8_t *actT, double lamT,
                     double *Theta) {
    /* Coordinate descent directly on the quadratic of Eq. (7):
     * along Theta_ij the change of g is mu b + 1/2 a mu^2 with
     * b = 2 Sxy_ij + 2 (Sxx Theta Sigma)_ij and a = 2 Sxx_ii Sigma_jj.
     * V = Theta Sigma is maintained (row i gains mu Sigma_j.), stored
     * transposed (Vt[j][k] = V[k][j]) so that the column of V read by every
     * coordinate is a contiguous row of Vt. */
    double *V = zalloc((size_t)(p * q)), *Vt = zalloc((size_t)(p * q));
    matmul(p, q, q, Theta, Sigma, V);
    for (int64_t k = 0; k < p; ++k)
        for (int64_t j = 0; j < q; ++j) Vt[IDX(j, k, p)] = V[IDX(k, j, q)];
    free(V);
    for (int64_t i = 0; i < p; ++i) {
        for (int64_t j = 0; j < q; ++j) {
            if (!actT[IDX(i, j, q)]) continue;
            double a = 2.0 * Sxx[IDX(i, i, p)] * Sigma[IDX(j, j, q)];
            if (!(a > 0.0)) continue;
            const double *Si = Sxx + IDX(i, 0, p), *Vcol_j = Vt + IDX(j, 0, p);
            double sv = 0.0;
            for (int64_t k = 0; k < p; ++k) sv += Si[k] * Vcol_j[k];
            double b = 2.0 * Sxy[IDX(i, j, q)] + 2.0 * sv;
            double c = Theta[IDX(i, j, q)];
            double z = soft_threshold(c - b / a, lamT / a);
            double mu = z - c;
            if (mu == 0.0) continue;
            Theta[IDX(i, j, q)] = z;
            const double *Sj = Sigma + IDX(j, 0, q);
            for (int64_t k = 0; k < q; ++k) Vt[IDX(k, i, p)] += mu * Sj[k];
        }
    }
    free(Vt);
}

/* l1 norm of the minimum-norm subgradient of f (stopping rule, Sec. 5.1). */
static double min_norm_subgrad_l1(size_t count, const double *G, const double *X,
                                  double lam) {
    double s = 0.0;
    for (size_t k = 0; k < count; ++k) {
        double g = G[k];
        if (X[k] != 0.0) {
            s += fabs(g + (X[k] > 0.0 ? lam : -lam));
        } else {
            double m = fabs(g) - lam;
            if (m > 0.0) s += m;
        }
    }
    return s;
}

static int64_t count_nonzero(size_t count, const double *A) {
    int64_t c = 0;
    for (size_t k = 0; k < count; ++k) c += (A[k] != 0.0);
    return c;
}

static int64_t count_mask(size_t count, const uint8_t *m) {
    int64_t c = 0;
    for (size_t k = 0; k < count; ++k) c += m[k];
    return c;
}

int orc_solve(int64_t n, int64_t p, int64_t q, const double *X, const double *Y,
              double lamL, double lamT, double tol, int max_iter, int stall_iters,
              int lambda_passes, int warm, double *Lambda, double *Theta, int *iters,
              double *f_final, orc_trace *trace) {
    size_t qq = (size_t)(q * q), pq = (size_t)(p * q);
    double *Sxx = zalloc((size_t)(p * p)), *Sxy = zalloc(pq), *Syy = zalloc(qq);
    double *L = zalloc(qq), *Sigma = zalloc(qq), *Psi = zalloc(qq), *M = zalloc(qq);
    double *GL = zalloc(qq), *GT = zalloc(pq), *D = zalloc(qq);
    uint8_t *actL = (uint8_t *)calloc(qq ? qq : 1, 1), *actT = (uint8_t *)calloc(pq ? pq : 1, 1);
    if (!actL || !actT) abort();
    orc_stats(n, p, q, X, Y, Sxx, Sxy, Syy);
    if (!warm) {                                  /* Algorithm 1: Theta = 0, Lambda = I */
        memset(Lambda, 0, sizeof(double) * qq);
        memset(Theta, 0, sizeof(double) * pq);
        for (int64_t i = 0; i < q; ++i) Lambda[IDX(i, i, q)] = 1.0;
    }
    int status = ORC_MAXITER, stalled = 0, t = 0;
    double sg_best = INFINITY, f_prev = INFINITY, f = 0.0;
    for (t = 0;; ++t) {
        if (orc_cholesky(q, Lambda, L) != ORC_OK) {
            status = ORC_NOTPD;
            break;
        }
        orc_inverse_from_cholesky(q, L, Sigma);
        gradient_given_sigma(p, q, Sxx, Sxy, Syy, Theta, Sigma, GL, GT, Psi, M);
        f = objective_from_parts(p, q, Sxy, Syy, Lambda, Theta, Sigma, M,
                                 logdet_from_cholesky(q, L), lamL, lamT);
        double sg = min_norm_subgrad_l1(qq, GL, Lambda, lamL) +
                    min_norm_subgrad_l1(pq, GT, Theta, lamT);
        double l1 = l1_norm(qq, Lambda) + l1_norm(pq, Theta);
        orc_active_sets(p, q, GL, GT, Lambda, Theta, lamL, lamT, actL, actT);
        if (trace) {
            trace->f[t] = f;
            trace->subgrad[t] = sg;
            trace->l1[t] = l1;
            trace->alpha[t] = NAN;
            trace->mL[t] = count_mask(qq, actL);
            trace->mT[t] = count_mask(pq, actT);
            trace->nnzL[t] = count_nonzero(qq, Lambda);
            trace->nnzT[t] = count_nonzero(pq, Theta);
            trace->ls_trials[t] = 0;
        }
        if (sg < tol * l1) {
            status = ORC_OK;
            break;
        }
        if (stall_iters > 0) {             /* neither f nor the subgradient moves */
            int no_progress = (sg >= sg_best) && (f >= f_prev - 1e-15 * fabs(f_prev));
            stalled = no_progress ? stalled + 1 : 0;
            if (stalled >= stall_iters) {
                status = ORC_STALLED;
                break;
            }
        }
        sg_best = sg < sg_best ? sg : sg_best;
        f_prev = f;
        if (t >= max_iter) {
            status = ORC_MAXITER;
            break;
        }
        /* Lambda step: Newton direction by one CD pass, then Armijo line search. */
        orc_lambda_direction(q, Sigma, Psi, GL, Lambda, actL, lamL, lambda_passes, D);
        double alpha = 0.0, fa = f;
        int trials = 0;
        orc_line_search(p, q, Sxx, Sxy, Syy, Lambda, Theta, D, GL, lamL, lamT, f, 0.5, 1e-3,
                        30, &alpha, &fa, &trials);
        if (trace) {
            trace->alpha[t] = alpha;
            trace->ls_trials[t] = trials;
        }
        /* Theta step with Sigma of the updated Lambda, same active set. */
        if (orc_cholesky(q, Lambda, L) != ORC_OK) {
            status = ORC_NOTPD;
            break;
        }
        orc_inverse_from_cholesky(q, L, Sigma);
        orc_theta_sweep(p, q, Sxx, Sxy, Sigma, actT, lamT, Theta);
    }
    *iters = t;
    *f_final = f;
    free(Sxx);
    free(Sxy);
    free(Syy);
    free(L);
    free(Sigma);
    free(Psi);
    free(M);
    free(GL);
    free(GT);
    free(D);
    free(actL);
    free(actT);
    return status;
}
