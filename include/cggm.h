/*
 * cggm.h -- C ABI of the MI355X (gfx950) alternating Newton coordinate descent
 * solver for the l1-regularized conditional Gaussian graphical model (CGGM).
 *
 * Problem (McCarter & Kim, AISTATS 2016, Sec. 2.1, Eq. (1)): given X (n x p)
 * and Y (n x q), minimise over symmetric positive definite Lambda (q x q) and
 * Theta (p x q)
 *
 *   f(Lambda, Theta) = -log det Lambda + tr(Syy Lambda) + 2 tr(Sxy^T Theta)
 *                      + tr(Lambda^{-1} Theta^T Sxx Theta)
 *                      + lamL ||Lambda||_1 + lamT ||Theta||_1
 *
 * with Sxx = X^T X / n, Sxy = X^T Y / n, Syy = Y^T Y / n (uncentred), and the
 * l1 norms elementwise over all entries (diagonal and both triangles).
 *
 * Conventions for every entry point:
 *   - All matrices are dense, row-major, contiguous, in DEVICE memory of the
 *     current HIP device, unless a parameter says "host"; float64, except the
 *     inputs X and Y, whose element type is the `dtype` argument (CGGM_F64 or
 *     CGGM_F32).
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     is ordered on it.  Entry points that return host scalars synchronise it.
 *   - Input pointers are only read during the call and never retained.
 *   - Return value: CGGM_OK (0), a warning (> 0: results are valid) or an error
 *     (< 0: outputs are left untouched).  cggm_last_error() gives a message for
 *     the last failing call on the calling thread.
 *   - No entry point throws.  The solve entry points (and cggm_sigma_columns)
 *     allocate their device workspace per call with hipMalloc and free it
 *     before returning; the request server allocates one device pool when it
 *     is created and carves every request's workspace out of it;
 *     cggm_objective_noalloc uses a static device array and allocates
 *     nothing; cggm_partition_graph works in host memory only.
 */
#ifndef CGGM_H
#define CGGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define CGGM_OK 0
#define CGGM_MAXITER 1        /* warning: iteration cap reached, result valid   */
#define CGGM_STALLED 2        /* warning: stopped because neither f nor the
                                 subgradient improved for options.stall_iters
                                 iterations (the rounding floor of f) before the
                                 stopping rule was met; result valid           */
#define CGGM_EINVAL (-1)      /* bad size, NULL pointer, non-finite value       */
#define CGGM_ENOTPD (-2)      /* Lambda (given or warm start) not pos. definite */
#define CGGM_ELINESEARCH (-3) /* no Armijo step found (last iterate returned)   */
#define CGGM_ENOMEM (-4)      /* workspace over budget or hipMalloc failed      */
#define CGGM_EHIP (-5)        /* a HIP runtime call failed                      */
#define CGGM_ECAPACITY (-6)   /* problem larger than a server's device pool or
                                 the static scratch of cggm_objective_noalloc  */

/* ---- element type of the inputs X and Y --------------------------------
 * CGGM_F32 inputs are widened exactly to FP64 copies in the workspace (8 (np + nq)
 * more bytes); every computation runs as for CGGM_F64 inputs holding the same
 * values.  The parameters Lambda and Theta are always FP64. */
#define CGGM_F64 0
#define CGGM_F32 1

/* ---- coordinate-descent sweep schedules ------------------------------ */
#define CGGM_SWEEP_TILED 0      /* conflict-free parallel tile waves (default)   */
#define CGGM_SWEEP_SEQUENTIAL 1 /* one coordinate at a time in lexicographic
                                   order: the order of the paper's Algorithm 1
                                   and of the CPU reference                      */

/* ---- arithmetic ---------------------------------------------------------
 * FP64: every step in FP64.
 * MIXED (problems with q >= options.mixed_min_q; smaller ones run in FP64):
 *   while the subgradient is above 1e-4 of the stopping scale
 *   (||Lambda||_1 + ||Theta||_1), the coordinate-descent sweeps (Sec. 3.1,
 *   3.2) stream FP32 copies of Sigma, Psi, Sigma + Psi and Sxx and maintain
 *   U = D Sigma and V = Theta Sigma in FP32, with their products on the FP32
 *   matrix cores, and V is formed from three-piece BF16 splits of Theta and
 *   Sigma on the BF16 matrix cores with FP32 accumulation; afterwards the
 *   sweeps run in FP64.  The Cholesky factor, log det, Sigma, Psi, both
 *   gradients, the screen, the stopping rule, the objective, the line search
 *   and the coordinate updates themselves stay FP64, so the Armijo test and
 *   the fixed point of the iteration are those of the FP64 mode. */
#define CGGM_PRECISION_FP64 0
#define CGGM_PRECISION_MIXED 1

/* One record per outer iteration (Algorithm 1), filled when options.trace is
 * non-NULL.  Values describe the iterate at the top of iteration `iter`. */
typedef struct {
    int iter;
    int ls_trials;        /* Cholesky trials in the line search                 */
    int sweep_fallbacks;  /* sweeps redone by the descent guards               */
    int sweep_split;      /* waves run as 2^(x & 255) (Lambda) and 2^(x >> 8)
                             (Theta) sub-waves in this iteration              */
    double f;             /* objective at the top of the iteration (FP64)       */
    double subgrad_l1;    /* l1 norm of the minimum-norm subgradient            */
    double l1;            /* ||Lambda||_1 + ||Theta||_1                          */
    double alpha;         /* accepted Lambda step size (0: no step)             */
    int64_t m_Lambda;     /* |S_Lambda| (upper triangle incl. diagonal)         */
    int64_t m_Theta;      /* |S_Theta|                                          */
    int64_t nnz_Lambda;   /* nonzeros of Lambda (both triangles)                */
    int64_t nnz_Theta;    /* nonzeros of Theta                                  */
    double t_end_ms;      /* wall time from the start of the solve to the end
                             of this record's top-of-iteration evaluation       */
    double ms_gradient;   /* products, gradients, screen, objective             */
    double ms_lambda_cd;  /* Lambda coordinate-descent sweep                     */
    double ms_line_search;/* line search incl. the accepted factor's inverse    */
    double ms_theta_cd;   /* V = Theta Sigma and the Theta sweep                 */
    double delta;         /* tr(G_Lambda D) + lamL (|Lambda + D|_1 - |Lambda|_1)
                             of the direction the line search took              */
} cggm_trace_entry;

/* Launch statistics of the coordinate-descent sweeps, filled when
 * options.kstats is non-NULL.  Each wave of a sweep runs three kernels
 * (stage 0: gradient snapshot products, 1: in-tile Gauss-Seidel, 2: update of
 * the maintained product).  Durations come from HIP events recorded on the
 * solve's stream around every launch; bytes and flops are the algorithmic
 * traffic and arithmetic of the tiles that had active coordinates (operand
 * slabs of the snapshot; the tile's Sigma / Psi / Sxx blocks, gradient and
 * parameter reads and writes; the rows of Sigma read and of U or V updated),
 * counted on the device.  Index [0] is the Lambda sweep, [1] the Theta sweep. */
typedef struct {
    int64_t waves[2];           /* waves run (kernel triples)                      */
    int64_t tiles[2];           /* tiles processed (with active coordinates)       */
    double ms[2][3];            /* summed launch durations per stage               */
    double bytes[2][3];         /* summed algorithmic bytes per stage              */
    double flops[2][3];         /* summed algorithmic flops per stage              */
} cggm_kernel_stats;

typedef struct {
    int max_iter;          /* outer iterations (default 500)                   */
    int max_ls;            /* line-search trials (default 30)                  */
    double ls_beta;        /* step shrink factor (default 0.5)                 */
    double ls_sigma;       /* Armijo sufficient-decrease constant (1e-3)       */
    int stall_iters;       /* stop after this many iterations without progress
                              in f or the subgradient (default 3; 0 = off)     */
    int sweep;             /* CGGM_SWEEP_TILED or CGGM_SWEEP_SEQUENTIAL        */
    int tile;              /* CD tile edge for CGGM_SWEEP_TILED (0 = default)  */
    int lambda_passes;     /* CD passes of the Lambda direction over S_Lambda
                              per iteration (Sec. 3 makes one); 0 (default):
                              4 when n >= q / 4, else 6 -- with fewer samples
                              Syy has low rank and the direction needs more
                              passes                                          */
    int precision;         /* CGGM_PRECISION_FP64 (default) or
                              CGGM_PRECISION_MIXED                             */
    int mixed_min_q;       /* CGGM_PRECISION_MIXED applies to problems with
                              q >= this (default 4096; 0 = always); smaller
                              ones run in FP64.  Below it the sweeps are bound
                              by the latency of small launches and
                              Gauss-Seidel chains, not by HBM, and the extra
                              conversions and split products only cost time
                              (at q = 2000 the mixed mode gained nothing; at
                              q = 20000 it takes an outer iteration from
                              6.9 s to 4.3 s on one MI355X)                   */
    size_t workspace_budget;   /* bytes of device workspace allowed (0 = any)  */
    const double *warm_Lambda; /* device q x q start (NULL = identity)         */
    const double *warm_Theta;  /* device p x q start (NULL = zero)             */
    cggm_trace_entry *trace;   /* host array of trace_cap records, or NULL     */
    int trace_cap;
    int trace_len;             /* out: records written                          */
    cggm_kernel_stats *kstats; /* out: CD sweep kernel statistics, or NULL       */
    int theta_passes;      /* CD passes of the Theta step over S_Theta per
                              iteration (Sec. 3.2 makes one; default 1); the
                              passes share Sigma and the active set          */
    int split_level;       /* tiled sweeps: each wave starts as 2^split_level
                              sub-waves run one after another (0..6, default
                              0: whole waves)                                 */
    int split_adapt;       /* 1 (default): the descent guards and the step
                              size move the level (see cggm_solve); 0: the
                              level stays at split_level and a failing sweep
                              is redone with one tile per wave               */
    int blockwise;         /* 1: block-wise Theta statistics (Sec. 4.2 of the
                              paper, Algorithm 2): the p x p matrix Sxx is
                              never formed; the Theta sweep runs by groups of
                              consecutive row tiles and forms the Sxx columns
                              of one group at a time from X (X^T X[:, group]
                              / n on the matrix cores) into a slab of at most
                              sxx_cache_bytes, skipping groups with no active
                              coordinate.  Results are those of the dense
                              mode up to the order of the tiles (with one
                              group, bit for bit).  Default 0.               */
    size_t sxx_cache_bytes;/* device bytes of that slab (0 = 2 GiB); at least
                              one row tile (64 p doubles) is always held     */
    int graphs;            /* 1: the kernel launches of each tiled sweep are
                              captured once into a HIP graph and replayed on
                              later sweeps with the same schedule, buffers,
                              penalty and precision (fewer host launches for
                              small problems; results identical).  Not with
                              kstats, and not for the block-wise Theta sweep
                              (it decides on the host which groups to form).
                              Default 0; the request server sets it.          */
} cggm_options;

/* Fill `opt` with the defaults above. */
void cggm_default_options(cggm_options *opt);

/* Device bytes cggm_solve would allocate for this shape with default options
 * and FP64 inputs (the footprint the workspace_budget option is compared
 * against; FP32 inputs add 8 (n p + n q) bytes, rounded up to 256 per array). */
size_t cggm_solve_workspace_bytes(int64_t n, int64_t p, int64_t q);

/* The same for the given options (NULL = defaults; the mixed mode needs more);
 * 0 for invalid sizes or options. */
size_t cggm_workspace_bytes(int64_t n, int64_t p, int64_t q, const cggm_options *opt);

typedef struct cggm_result cggm_result;   /* opaque, owns device CSR arrays */

/*
 * Alternating Newton coordinate descent (Algorithm 1): from Lambda = I,
 * Theta = 0 (or the warm start), each outer iteration
 *   1. factors Lambda = L L^T, forms Sigma = Lambda^{-1}, log det Lambda,
 *      R = X Theta Sigma, Psi = R^T R / n and the gradients of Eq. (3),
 *   2. screens the active sets |grad| > lambda or param != 0 (Sec. 2.2),
 *   3. finds the generalized Newton direction D of Eq. (6) by
 *      options.lambda_passes coordinate-descent passes over S_Lambda (the
 *      paper makes one), maintaining U = D Sigma,
 *   4. takes the Armijo step Lambda + alpha D that keeps Lambda positive
 *      definite (Algorithm 1, line search),
 *   5. minimises Eq. (7) over Theta by one coordinate-descent pass over
 *      S_Theta, maintaining V = Theta Sigma (Sec. 3.2).
 * The passes run as waves of 64 x 64 tiles whose maintained-product rows are
 * disjoint (exact Gauss-Seidel inside a tile, concurrent across the tiles of
 * a wave), or one coordinate at a time with CGGM_SWEEP_SEQUENTIAL.  A
 * direction with no descent or for which the line search finds no Armijo
 * step, or a Theta pass that raises f, is redone: in FP64 after a
 * mixed-precision pass, else with each wave split into twice as many
 * sub-waves (up to 64), else one tile per wave; a Lambda step shrunk below
 * 1/8 by the line search also doubles the split, three full steps in a row
 * (any step below 1 restarts the count) halve it.
 * It stops when ||grad^S||_1 < tol (||Lambda||_1 + ||Theta||_1) (the paper's
 * stopping rule of Sec. 5.1 with 0.01 replaced by tol; CGGM_OK), when the
 * iterate stops moving (stall_iters; CGGM_STALLED), or after max_iter
 * iterations (CGGM_MAXITER).
 *
 * X: n x p, Y: n x q (device) of element type dtype (CGGM_F64 or CGGM_F32).
 * lamL, lamT >= 0.  On success *out receives a
 * result handle (free with cggm_result_free).  The call is blocking: it
 * synchronises `stream` to take the line-search and stopping decisions.
 * Errors: CGGM_EINVAL (n, p, q < 1, NULL pointers, negative or non-finite
 * lambda/tol, non-finite X or Y), CGGM_ENOTPD (warm_Lambda not positive
 * definite), CGGM_ENOMEM (footprint over workspace_budget or out of memory),
 * CGGM_EHIP.  CGGM_ELINESEARCH is returned with a valid result when no step
 * satisfying the Armijo rule exists for a descent direction.
 */
int cggm_solve(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
               double lamL, double lamT, double tol, cggm_options *opt,
               cggm_result **out, void *stream);

/*
 * Regularisation path: the solves of cggm_solve at the npath penalty pairs
 * (lamL[k], lamT[k]) (host arrays), taken in order, each starting from the
 * previous point's result (warm starts; the paper solves one penalty pair at a
 * time, this is the batched form of its Algorithm 1); the first point starts
 * from options.warm_* or from Lambda = I, Theta = 0.  The statistics Sxx, Sxy, Syy are formed once and
 * the workspace (Sigma, the factor, the maintained products) stays resident
 * between points.  Point k's result is bit-for-bit the result of cggm_solve at
 * (lamL[k], lamT[k]) warm-started from point k-1's Lambda and Theta.
 * out: host array of npath handles, all filled unless the return value is an
 * error other than CGGM_ELINESEARCH (then none are).  Returns the first
 * negative status of a point, else CGGM_MAXITER if a point reached the cap,
 * else CGGM_STALLED if a point stalled, else CGGM_OK; each point's own status
 * is in cggm_result_info.  Trace records
 * of all points are appended in order (iter restarts at 0 for each point).
 */
int cggm_solve_path(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                    int npath, const double *lamL, const double *lamT, double tol,
                    cggm_options *opt, cggm_result **out, void *stream);

/* Scalars of a result: nonzeros of Lambda (both triangles) and Theta, the
 * number of outer iterations, the final objective and the solve status. */
int cggm_result_info(const cggm_result *res, int64_t *nnz_Lambda, int64_t *nnz_Theta,
                     int *iters, double *f, int *status);

/* Copy the CSR form of Lambda (q rows, full symmetric) and Theta (p rows) into
 * caller buffers: rowptr (rows + 1 int64), col (nnz int32), val (nnz float64).
 * to_host != 0: buffers are host memory; otherwise device memory.  Any of the
 * six pointers may be NULL to skip that array. */
int cggm_result_copy(const cggm_result *res, int64_t *L_rowptr, int32_t *L_col,
                     double *L_val, int64_t *T_rowptr, int32_t *T_col, double *T_val,
                     int to_host);

/* Copy the dense Lambda (q x q) and Theta (p x q) into caller buffers. */
int cggm_result_dense(const cggm_result *res, double *Lambda, double *Theta, int to_host);

void cggm_result_free(cggm_result *res);

/*
 * Objective f(Lambda, Theta) of Eq. (1) at dense device Lambda (q x q,
 * symmetric) and Theta (p x q); *f_out is a host double.  Returns CGGM_ENOTPD
 * when Lambda is not positive definite (f is +infinity there).
 */
int cggm_objective(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                   const double *Lambda, const double *Theta, double lamL, double lamT,
                   double *f_out, void *stream);

/*
 * Allocation-free form of cggm_objective, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, result and errors as
 * cggm_objective; it calls no hipMalloc, hipFree or allocating library
 * routine.  Its workspace -- three n x q arrays (X Theta, its transpose,
 * Y Lambda), the Cholesky factor (q x q), the inverted 64 x 64 diagonal
 * blocks (64 ceil(q / 64) x 64), about 5 KB of reduction scratch and, for
 * CGGM_F32 inputs, the FP64 copies of X and Y, 8-byte words, each array
 * rounded up to 256 bytes -- comes from a static device
 * array of CGGM_NOALLOC_SCRATCH_BYTES (64 MiB) that every device the library
 * runs on holds until the process ends.  A shape whose workspace exceeds it
 * returns CGGM_ECAPACITY before any device work: q = n = 1000 (31 MiB),
 * q = 1500 with n = 1000 (52 MiB) and q = 2000 with n = 500 (54 MiB) fit,
 * q = 2000 with n = 1000 (77 MiB) does not.  All calls on one device
 * share that device's array: calls that overlap on one device (from several
 * host threads, or on several streams) race and must be serialised by the
 * caller.  The call synchronises `stream` to read f back.
 */
#define CGGM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int cggm_objective_noalloc(const void *X, const void *Y, int64_t n, int64_t p, int64_t q,
                           int dtype, const double *Lambda, const double *Theta, double lamL,
                           double lamT, double *f_out, void *stream);

/*
 * Tile-edge autotuner for problems of shape (n, p, q): runs a synthetic
 * problem of that shape (X, Y standard normal from a deterministic
 * counter-based generator, lambda = 0.02, near-dense active sets) with the
 * options `opt` (NULL = defaults) and each candidate tile edge 16, 32, 64 for
 * one warm-up and `iters` (1..50) timed outer iterations from Lambda = I,
 * Theta = 0, twice per edge in the order 64, 32, 16, 16, 32, 64, and writes
 * to *tile (host) the edge with the shortest time per iteration (the better
 * of its two runs), where 64 stays unless a smaller edge is at least 5%
 * faster, and, when `ms` is not NULL, the three times in milliseconds (host,
 * 3 doubles, for 16, 32, 64).  Pass the edge as options.tile (or a request's tile) for
 * problems of about that shape.  The choice changes the order of the
 * coordinate updates, hence the iterates, not the optimum.  Allocates its
 * own inputs and one solve workspace at a time; blocking.
 */
int cggm_autotune_tile(int64_t n, int64_t p, int64_t q, const cggm_options *opt, int iters,
                       int *tile, double *ms, void *stream);

/*
 * One generalized Newton direction of the Lambda step (Algorithm 1, Eq. (6))
 * at a given point, as cggm_solve computes it: at dense device Lambda
 * (q x q, symmetric positive definite) and Theta (p x q) it forms Sigma, Psi
 * and the gradients (Eq. (3)), screens the active set (Sec. 2.2) and makes
 * opt->lambda_passes coordinate-descent passes over it from D = 0 in the
 * schedule and precision of `opt` (NULL = defaults; tiled sweeps at
 * opt->split_level, without the descent guards).  Outputs (caller device
 * buffers, NULL skips): D (q x q, both triangles), U = D Sigma as maintained
 * by the passes (q x q; FP32 arithmetic in the mixed mode, widened), and
 * V = Theta Sigma as the Theta step forms it (p x q: a sparse-by-dense FP64
 * product when fewer than 2% of Theta's entries are nonzero, else a dense
 * FP64 product, or split-BF16 products in the mixed mode; stored in FP32 in
 * the mixed mode).  For checking the steps of the solver against a
 * reference; allocates and frees a solve workspace.  Errors as cggm_solve,
 * CGGM_ENOTPD when Lambda is not positive definite.
 */
int cggm_lambda_direction(const void *X, const void *Y, int64_t n, int64_t p, int64_t q,
                          int dtype, const double *Lambda, const double *Theta, double lamL,
                          double lamT, const cggm_options *opt, double *D, double *U,
                          double *V, void *stream);

/*
 * Gradient of the smooth part g at (Lambda, Theta), Eq. (3):
 *   G_Lambda = Syy - Sigma - Psi      (q x q, Psi = Sigma Theta^T Sxx Theta Sigma)
 *   G_Theta  = 2 Sxy + 2 Sxx Theta Sigma   (p x q)
 * written to caller device buffers.  CGGM_ENOTPD if Lambda is not PD.
 */
int cggm_gradient(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                  const double *Lambda, const double *Theta, double *G_Lambda,
                  double *G_Theta, void *stream);

/*
 * Columns of Sigma = Lambda^{-1} by conjugate gradients, as the block-wise
 * method (Sec. 4.1) obtains the Sigma columns of a block: for each listed
 * column j it solves Lambda x = e_j, with Lambda sparse symmetric positive
 * definite, in O(m_Lambda) work per iteration and column; up to 64 columns
 * advance together (one sparse-by-dense product per iteration), larger lists
 * run in batches of 64.
 *   rowptr, col, val: Lambda in CSR with both triangles stored (device
 *     pointers; rowptr holds q + 1 int64 offsets starting at 0, col the int32
 *     column of each of the rowptr[q] entries, val their values).  rowptr is
 *     checked on the host and col on the device before any product: a
 *     decreasing rowptr or a column outside [0, q) gives CGGM_EINVAL.  The
 *     symmetry of Lambda is the caller's to guarantee.
 *   cols: host array of k column indices in [0, q) (repeats allowed).
 *   tol: a column stops once its residual norm ||e_j - Lambda x|| is at most
 *     tol (the right-hand side has unit norm, so tol is relative); tol >= 0.
 *   max_iter: iterations per batch, >= 1 (checked every 8 iterations, so a
 *     batch may run up to 7 iterations past convergence, without changing
 *     its converged columns).
 *   Sigma_C: caller device buffer of q x k doubles, row-major: column t is
 *     Sigma's column cols[t].
 *   iters, resid (host, may be NULL): the most iterations a batch ran, and
 *     the largest final residual norm over the columns.
 * Returns CGGM_OK when every column reached tol, CGGM_MAXITER (result valid)
 * when some did not within max_iter, CGGM_ENOTPD when a search direction met
 * a curvature p^T Lambda p that is not positive (Lambda not positive
 * definite), CGGM_EINVAL, CGGM_ENOMEM (the call allocates 2.5 KiB per row
 * of Lambda plus 0.5 MiB, freed before it returns) or CGGM_EHIP.  Work is ordered
 * on `stream` and the call returns when it is done.
 */
int cggm_sigma_columns(const int64_t *rowptr, const int32_t *col, const double *val,
                       int64_t q, const int32_t *cols, int64_t k, double tol, int max_iter,
                       double *Sigma_C, int *iters, double *resid, void *stream);

/*
 * Balanced k-way partition of a graph minimising the number of cut edges,
 * for the column blocks of the block-wise method: Sec. 4.1 clusters the
 * graph of Lambda's active set so that few active entries fall in
 * off-diagonal blocks, and Sec. 4.2 clusters the columns of Theta through
 * the graph of the nonzeros of Theta^T Theta; this takes the place of the
 * external partitioning library the paper uses.  Host memory, computed on
 * the host (recursive bisection: greedy growing from a peripheral vertex,
 * then Fiduccia-Mattheyses refinement); deterministic.
 *   n: vertices, 1 <= n < 2^31.
 *   rowptr (n + 1 int64, starting at 0, not decreasing), col (rowptr[n]
 *     int32 in [0, n)): the adjacency pattern in CSR.  The graph is the
 *     undirected union of the listed pairs: (u, v) and (v, u) are one edge,
 *     repeats and self loops are ignored, so a triangle or a full symmetric
 *     pattern may be given.
 *   nparts: 1 <= nparts <= n.
 *   imbalance >= 0: every part gets at least one vertex and at most
 *     max(ceil(n / nparts), floor((1 + imbalance) n / nparts)).
 *   part (host, n int32): the part of each vertex, in [0, nparts).
 *   cut (host, may be NULL): the number of edges between different parts.
 * Returns CGGM_OK or CGGM_EINVAL (bad sizes or pattern; part untouched).
 */
int cggm_partition_graph(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t nparts,
                         double imbalance, int32_t *part, int64_t *cut);

/* ---- request server (continuous batching on one GPU) --------------------
 *
 * Solves regularisation paths of many independent problems concurrently on
 * one device.  The server owns `slots` worker threads, each with its own HIP
 * stream (default priority), and one device pool of pool_bytes.  A submitted
 * request waits in a queue until a slot is idle and the pool has a free
 * block for its workspace (cggm_workspace_bytes of its shape and options);
 * it then holds that block until its path is done, so requests that arrive
 * while others run are admitted as slots and memory free up, and their
 * kernels overlap on the device.  Admission is first come, first served,
 * except that a later request that fits may pass a waiting head that does
 * not fit, at most max_bypass times in a row for the same head.  A request's
 * results do not depend on what else runs: the kernels are deterministic and
 * every request has its own workspace and stream.
 */
typedef struct cggm_server cggm_server;

typedef struct {
    const void *X, *Y;        /* device, n x p and n x q of element type dtype;
                                 valid until the request completes
                                 (cggm_server_wait returned)                     */
    int64_t n, p, q;
    int npath;                /* >= 1 penalty pairs                               */
    const double *lamL;       /* host, npath values (copied at submit)            */
    const double *lamT;       /* host, npath values (copied at submit)            */
    double tol;               /* stopping rule of cggm_solve                      */
    int precision;            /* CGGM_PRECISION_*                                 */
    int max_iter;             /* per path point; 0 = default                      */
    int lambda_passes;        /* 0 = default                                      */
    int mixed_min_q;          /* as cggm_options.mixed_min_q; < 0 = default      */
    double *Lambda_out;       /* device npath x q x q, or NULL                    */
    double *Theta_out;        /* device npath x p x q, or NULL                    */
    int dtype;                /* CGGM_F64 (0) or CGGM_F32                          */
    int tile;                 /* CD tile edge (0 = default; cggm_autotune_tile)   */
} cggm_request;

typedef struct {
    int status;               /* as cggm_solve_path, or the error of the request  */
    int slot;                 /* worker that ran it                               */
    int iters_total;          /* outer iterations over the path                   */
    int _pad;
    double t_submit_ms;       /* times since the server was created               */
    double t_admit_ms;
    double t_done_ms;
    size_t footprint;         /* pool bytes the request held                      */
} cggm_request_info;

typedef struct {
    int64_t submitted, completed, rejected;
    int max_running;          /* most requests on the device at once              */
    int _pad;
    size_t pool_bytes;
    size_t peak_bytes_in_use; /* most pool bytes held at once                     */
} cggm_server_stats;

/* Create a server on the current device.  slots >= 1; max_bypass >= 0.
 * Errors: CGGM_EINVAL, CGGM_ENOMEM (the pool cannot be allocated), CGGM_EHIP. */
int cggm_server_create(int slots, size_t pool_bytes, int max_bypass, cggm_server **out);

/* Queue a request; *ticket identifies it.  Returns at once.  Errors:
 * CGGM_EINVAL (bad sizes, NULL pointers, penalties, options), CGGM_ECAPACITY
 * (its workspace exceeds the whole pool: it could never be admitted). */
int cggm_server_submit(cggm_server *srv, const cggm_request *req, int64_t *ticket);

/* Block until the request is done; fill *info (may be NULL) and, when not
 * NULL, the host arrays f (npath objectives) and iters (npath counts).  Each
 * ticket is waited for once; the request's memory on the server is released
 * then.  Returns the request's status (or CGGM_EINVAL for an unknown ticket). */
int cggm_server_wait(cggm_server *srv, int64_t ticket, cggm_request_info *info, double *f,
                     int *iters);

int cggm_server_stats_get(cggm_server *srv, cggm_server_stats *st);

/* Finish every queued and running request, stop the workers, free the pool.
 * Requests not yet waited for are discarded. */
void cggm_server_destroy(cggm_server *srv);

/* Static text for a status code; thread-local text of the last error. */
const char *cggm_status_string(int status);
const char *cggm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CGGM_H */
