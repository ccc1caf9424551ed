/* Runs every entry point of the CPU oracle (oracle/cggm_oracle.c) on small
 * problems, for a build with AddressSanitizer and UndefinedBehaviorSanitizer:
 * out-of-bounds accesses, leaks and undefined arithmetic in the checker fail
 * the run.  The data are arbitrary (a xorshift generator); the solve's result
 * is only checked for being finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cggm_oracle.h"

static unsigned long long rng_state = 88172645463325252ULL;
static double uniform(void) {               /* xorshift64, values in [-1, 1) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 4503599627370496.0 - 1.0;
}

static int run(int64_t n, int64_t p, int64_t q, int passes) {
    double *X = malloc(sizeof(double) * n * p), *Y = malloc(sizeof(double) * n * q);
    for (int64_t k = 0; k < n * p; ++k) X[k] = uniform();
    for (int64_t k = 0; k < n * q; ++k) Y[k] = uniform() + 0.3 * X[k % (n * p)];
    double *Sxx = malloc(sizeof(double) * p * p), *Sxy = malloc(sizeof(double) * p * q);
    double *Syy = malloc(sizeof(double) * q * q), *Lam = calloc(q * q, sizeof(double));
    double *Th = calloc(p * q, sizeof(double)), *GL = malloc(sizeof(double) * q * q);
    double *GT = malloc(sizeof(double) * p * q), *Sg = malloc(sizeof(double) * q * q);
    double *Ps = malloc(sizeof(double) * q * q), *D = malloc(sizeof(double) * q * q);
    double *L = malloc(sizeof(double) * q * q);
    uint8_t *aL = malloc(q * q), *aT = malloc(p * q);
    orc_stats(n, p, q, X, Y, Sxx, Sxy, Syy);
    for (int64_t i = 0; i < q; ++i) Lam[i * q + i] = 1.0;
    double f = 0.0;
    int bad = 0;
    bad |= orc_cholesky(q, Lam, L) != ORC_OK;
    orc_inverse_from_cholesky(q, L, Sg);
    bad |= orc_objective(p, q, Sxx, Sxy, Syy, Lam, Th, 0.1, 0.1, &f) != ORC_OK;
    bad |= orc_gradient(p, q, Sxx, Sxy, Syy, Lam, Th, GL, GT, Sg, Ps) != ORC_OK;
    orc_active_sets(p, q, GL, GT, Lam, Th, 0.1, 0.1, aL, aT);
    orc_lambda_direction(q, Sg, Ps, GL, Lam, aL, 0.1, passes, D);
    double alpha = 0.0, fa = 0.0;
    int trials = 0;
    (void)orc_line_search(p, q, Sxx, Sxy, Syy, Lam, Th, D, GL, 0.1, 0.1, f, 0.5, 1e-3, 30, &alpha,
                          &fa, &trials);
    orc_theta_sweep(p, q, Sxx, Sxy, Sg, aT, 0.1, Th);
    /* a full solve with a trace */
    const int max_iter = 200;
    double *tf = malloc(sizeof(double) * (max_iter + 1) * 4);
    int64_t *ti = malloc(sizeof(int64_t) * (max_iter + 1) * 4);
    int *tl = malloc(sizeof(int) * (max_iter + 1));
    orc_trace tr = {tf, tf + (max_iter + 1), tf + 2 * (max_iter + 1), tf + 3 * (max_iter + 1),
                    ti, ti + (max_iter + 1), ti + 2 * (max_iter + 1), ti + 3 * (max_iter + 1),
                    tl};
    int iters = 0;
    int st = orc_solve(n, p, q, X, Y, 0.05, 0.08, 1e-8, max_iter, 3, passes, 0, Lam, Th, &iters,
                       &f, &tr);
    bad |= !(st == ORC_OK || st == ORC_STALLED || st == ORC_MAXITER) || !isfinite(f);
    /* a non-positive-definite Lambda is reported, not used */
    memset(Lam, 0, sizeof(double) * q * q);
    bad |= orc_objective(p, q, Sxx, Sxy, Syy, Lam, Th, 0.1, 0.1, &f) != ORC_NOTPD;
    free(X), free(Y), free(Sxx), free(Sxy), free(Syy), free(Lam), free(Th), free(GL), free(GT);
    free(Sg), free(Ps), free(D), free(L), free(aL), free(aT), free(tf), free(ti), free(tl);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= run(30, 7, 5, 1);
    bad |= run(6, 9, 4, 2);      /* fewer samples than inputs */
    bad |= run(40, 1, 1, 1);
    bad |= run(20, 70, 65, 1);   /* large enough for the huge-page allocation path */
    printf(bad ? "oracle sanitize: FAILED\n" : "oracle sanitize: ok\n");
    return bad;
}
