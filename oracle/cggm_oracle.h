/*
 * cggm_oracle.h -- plain FP64 CPU reference of alternating Newton coordinate
 * descent (ANCD) for the l1-regularized conditional Gaussian graphical model.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the GPU library never does, and the two share no
 * code.  All matrices are dense, row-major, float64.  Sizes are int64.
 *
 * Notation (paper, Sec. 2.1): X is n x p, Y is n x q; Sxx = X^T X / n,
 * Sxy = X^T Y / n, Syy = Y^T Y / n; Lambda is q x q symmetric positive
 * definite, Theta is p x q; Sigma = Lambda^{-1}; Psi = Sigma Theta^T Sxx Theta Sigma.
 */
#ifndef CGGM_ORACLE_H
#define CGGM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define ORC_OK 0
#define ORC_MAXITER 1
#define ORC_STALLED 2
#define ORC_NOTPD (-2)

/* Sample covariances with the 1/n scaling and no centering (Sec. 2.1). */
void orc_stats(int64_t n, int64_t p, int64_t q, const double *X, const double *Y,
               double *Sxx, double *Sxy, double *Syy);

/* Dense Cholesky A = L L^T (L lower, upper part zeroed). Returns ORC_NOTPD if a
 * pivot is not strictly positive. */
int orc_cholesky(int64_t q, const double *A, double *L);

/* Sigma = (L L^T)^{-1} from a Cholesky factor. */
void orc_inverse_from_cholesky(int64_t q, const double *L, double *Sigma);

/* f(Lambda, Theta) of Eq. (1); ORC_NOTPD when Lambda is not positive definite. */
int orc_objective(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                  const double *Syy, const double *Lambda, const double *Theta,
                  double lamL, double lamT, double *f);

/* Gradient of the smooth part g, Eq. (3): G_Lambda = Syy - Sigma - Psi,
 * G_Theta = 2 Sxy + 2 Sxx Theta Sigma.  Sigma and Psi are also returned when
 * the pointers are non-NULL. */
int orc_gradient(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                 const double *Syy, const double *Lambda, const double *Theta,
                 double *GL, double *GT, double *Sigma, double *Psi);

/* Active sets (Sec. 2.2): S_Lambda over the upper triangle i <= j, S_Theta over
 * all entries; an entry is active when |gradient| > lambda or the parameter is
 * nonzero.  Output masks are q x q and p x q bytes (1 = active). */
void orc_active_sets(int64_t p, int64_t q, const double *GL, const double *GT,
                     const double *Lambda, const double *Theta, double lamL,
                     double lamT, uint8_t *actL, uint8_t *actT);

/* Coordinate descent for the generalized Newton direction D of Eq. (6):
 * `passes` passes over S_Lambda, each in lexicographic (i, j) order, from
 * D = 0, maintaining U = D Sigma (Sec. 3 makes a single pass).  D is written
 * as a full symmetric q x q matrix. */
void orc_lambda_direction(int64_t q, const double *Sigma, const double *Psi,
                          const double *GL, const double *Lambda, const uint8_t *actL,
                          double lamL, int passes, double *D);

/* Armijo line search on Lambda + alpha D (Algorithm 1): updates Lambda in
 * place with the accepted step and returns alpha (0 when D is not a descent
 * direction or no trial was accepted). */
int orc_line_search(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                    const double *Syy, double *Lambda, const double *Theta,
                    const double *D, const double *GL, double lamL, double lamT,
                    double f0, double beta, double sigma, int max_ls,
                    double *alpha_out, double *f_out, int *trials_out);

/* One coordinate-descent pass over S_Theta for Eq. (7) in lexicographic order,
 * maintaining V = Theta Sigma; updates Theta in place. */
void orc_theta_sweep(int64_t p, int64_t q, const double *Sxx, const double *Sxy,
                     const double *Sigma, const uint8_t *actT, double lamT,
                     double *Theta);

/* Per-iteration record written by orc_solve (arrays of length max_iter + 1). */
typedef struct {
    double *f;          /* objective at the top of the iteration            */
    double *subgrad;    /* l1 norm of the minimum-norm subgradient           */
    double *l1;         /* ||Lambda||_1 + ||Theta||_1                          */
    double *alpha;      /* accepted Lambda step (NaN on the final record)      */
    int64_t *mL, *mT;   /* active-set sizes                                    */
    int64_t *nnzL, *nnzT;
    int *ls_trials;
} orc_trace;

/* Full ANCD (Algorithm 1) from Lambda = I, Theta = 0 (or the given start when
 * warm != 0).  Stops when ||grad^S||_1 < tol (||Lambda||_1 + ||Theta||_1)
 * (the paper's stopping rule with 0.01 replaced by tol), when for
 * stall_iters consecutive iterations (stall_iters > 0) f has not decreased by
 * more than its rounding error and that subgradient norm has not reached a new
 * minimum (the rounding floor), or after
 * max_iter iterations.  lambda_passes (>= 1) is the number of CD passes of
 * the Lambda direction per iteration.  Returns ORC_OK / ORC_STALLED / ORC_MAXITER; *iters is
 * the number of completed iterations; trace may be NULL. */
int orc_solve(int64_t n, int64_t p, int64_t q, const double *X, const double *Y,
              double lamL, double lamT, double tol, int max_iter, int stall_iters,
              int lambda_passes, int warm, double *Lambda, double *Theta, int *iters,
              double *f_final, orc_trace *trace);

#ifdef __cplusplus
}
#endif
#endif
