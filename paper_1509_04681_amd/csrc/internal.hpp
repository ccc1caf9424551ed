// internal.hpp -- host-side interfaces between the translation units of the
// gfx950 CGGM solver library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

#include "cggm.h"
#include "tile_rect.hpp"

namespace cggm {

// Internal error carried to the C ABI boundary, where it becomes a status code.
struct Failure : std::runtime_error {
    int code;
    Failure(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw Failure(code, msg); }

#define CGGM_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::cggm::fail(CGGM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CGGM_LAUNCH_CHECK() CGGM_HIP(hipGetLastError())

// ---------------------------------------------------------------- la.hip ---
enum { UPLO_FULL = 0, UPLO_LOWER = 1 };
enum { KRANGE_FULL = 0, KRANGE_FROM_ROW = 1 };

// C = alpha op(A) op(B) + beta C, all row-major FP64, op(X) = X or X^T.
// Output tiles are 128 x 128 when M, N and K are all >= 256, else 64 x 64.
// uplo = UPLO_LOWER computes only the output tiles on or below the diagonal
// (entries above the diagonal inside those tiles are written too).
// krange = KRANGE_FROM_ROW starts the inner sum of an output tile at k = its
// first row (for products whose A operand is zero above that row, as in
// L^{-T} L^{-1}).  C may alias A or B only when every output tile reads
// exactly the operand rows / columns it writes (one K chunk per tile row).
void gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
          int64_t ldc, int uplo = UPLO_FULL, int krange = KRANGE_FULL);

// Mirror the strict lower triangle of the q x q matrix A into its upper triangle.
void symmetrize_from_lower(hipStream_t s, int64_t q, double *A);

// A = I (q x q).
void set_identity(hipStream_t s, int64_t q, double *A);

// dst (cols x rows) = src^T (src rows x cols).
void transpose(hipStream_t s, int64_t rows, int64_t cols, const double *src, double *dst);

// Panel width of the blocked factorizations; `Wd` arrays hold the inverses
// of the diagonal PB x PB blocks of a Cholesky factor (diag_inv_count(q)
// doubles).
constexpr int PB = 64;
inline int64_t diag_inv_count(int64_t q) { return ((q + PB - 1) / PB) * PB * PB; }

// In-place blocked right-looking Cholesky of the lower triangle of A (q x q,
// ld = q): on return the lower triangle holds L with A = L L^T and Wd the
// inverses of its diagonal blocks.  *notpd_dev (device int) is set to 1 when a
// pivot is not strictly positive.
void cholesky_inplace(hipStream_t s, int64_t q, double *A, int *notpd_dev, double *Wd);

// Solve L Z = B in place (B is q x m, leading dimension ldb, L lower q x q
// with diagonal-block inverses Wd).  lower_rhs = true declares B lower
// triangular (B = I) so only the columns a lower-triangular solution can
// populate are touched.
void trsm_lower_left(hipStream_t s, int64_t q, const double *L, const double *Wd, double *B,
                     int64_t m, int64_t ldb, bool lower_rhs);

// Sigma = (L L^T)^{-1} from the Cholesky factor: W = L^{-1} (into `work`,
// q x q), then Sigma = W^T W (lower tiles, k from the row block) mirrored.
void spd_inverse_from_cholesky(hipStream_t s, int64_t q, const double *L, const double *Wd,
                               double *work, double *Sigma);

// Deterministic sums: each call reduces into `out[0..nv)` (device) through a
// fixed-size partials buffer (device, >= REDUCE_BLOCKS * 8 doubles).
constexpr int REDUCE_BLOCKS = 512;

// out[0] = 2 sum_i log L_ii; out[1] = 1 if some L_ii <= 0 or non-finite.
void reduce_logdet(hipStream_t s, int64_t q, const double *L, double *partials, double *out);

// out[0] = sum A_ij B_ij over `count` entries.
void reduce_dot(hipStream_t s, int64_t count, const double *A, const double *B,
                double *partials, double *out);

// Statistics of the top of an iteration over a matrix pair (G, P) with
// penalty lam (P = Lambda with G = G_Lambda and upper = 1, or P = Theta with
// G = G_Theta):
//   out[0] = sum_ij W_ij P_ij           (W = Syy or Sxy; tr(W^T P))
//   out[1] = ||P||_1
//   out[2] = l1 norm of the minimum-norm subgradient
//   out[3] = active count (|G| > lam or P != 0; upper triangle only if upper)
//   out[4] = nonzeros of P
void reduce_top_stats(hipStream_t s, int64_t rows, int64_t cols, const double *W,
                      const double *G, const double *P, double lam, int upper,
                      double *partials, double *out);

// Line-search quantities of a direction D:
//   out[0] = sum G_ij D_ij,   out[1] = sum (|Lambda + D| - |Lambda|)  (entrywise)
void reduce_direction(hipStream_t s, int64_t q, const double *G, const double *Lam,
                      const double *D, double *partials, double *out);

// Trial point: T = Lambda + alpha D written to `trial`; out[0] = tr(Syy T),
// out[1] = ||T||_1.
void build_trial(hipStream_t s, int64_t q, const double *Lam, const double *D, double alpha,
                 const double *Syy, double *trial, double *partials, double *out);

// Gradient assembly: GL = Syy - Sigma - Psi, SP = Sigma + Psi.
void assemble_lambda_gradient(hipStream_t s, int64_t q, const double *Syy,
                              const double *Sigma, const double *Psi, double *GL, double *SP);

// y = a x (count entries).
void scale_copy(hipStream_t s, int64_t count, double a, const double *x, double *y);

// y = (float)x elementwise (rows x cols, row lengths ldx and ldy >= cols; the
// columns [cols, ldy) of y are set to zero); y = v.
void to_f32(hipStream_t s, int64_t rows, int64_t cols, const double *x, int64_t ldx, float *y,
            int64_t ldy);
void fill_f32(hipStream_t s, int64_t count, float v, float *y);

// Set a device int to a value (a kernel, so the stream may be graph-captured).
void set_int(hipStream_t s, int *dst, int v);

// Count non-finite entries of x into out[0] (as a double).
void reduce_nonfinite(hipStream_t s, int64_t count, const double *x, double *partials,
                      double *out);

// ------------------------------------------------------------- mixed.hip ---
// Row length of the BF16 pieces of a matrix with `cols` columns (padded to the
// K step of the split product, the padding zero).
int64_t split3_stride(int64_t cols);

// The three BF16 pieces hi, mid, lo of X (rows x cols, leading dimension ldx):
// planes[t * rows * split3_stride(cols) + r * split3_stride(cols) + c].
void split3(hipStream_t s, int64_t rows, int64_t cols, const double *X, int64_t ldx,
            __bf16 *planes);

// C (M x N, FP64, leading dimension ldc) = A B^T from the pieces of A (M x K)
// and B (N x K), the six leading cross products on the BF16 matrix cores with
// FP32 accumulation.
void gemm_split3_nt(hipStream_t s, int64_t M, int64_t N, int64_t K, const __bf16 *Ap,
                    const __bf16 *Bp, double *C, int64_t ldc);
// The same with an FP32 result (the FP32 accumulators stored as they are).
void gemm_split3_nt(hipStream_t s, int64_t M, int64_t N, int64_t K, const __bf16 *Ap,
                    const __bf16 *Bp, float *C, int64_t ldc);

// ---------------------------------------------------------------- cd.hip ---

constexpr int LAMBDA_TILE = 64;   // tile edge of the Lambda CD tiles
constexpr int THETA_TILE = 64;    // tile edge of the Theta CD tiles

// Optional instrumentation of a wave: events recorded before the snapshot,
// the Gauss-Seidel and the update kernels and after the update, and device
// counters the Gauss-Seidel kernel adds each processed tile's algorithmic
// traffic to: [0] tiles, [1, 2] snapshot bytes / flops, [3, 4] Gauss-Seidel
// bytes / flops, [5, 6] update bytes / flops.
struct WaveProbe {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    unsigned long long *counters = nullptr;   // [8]
};

// Scratch of the split gradient snapshots: partial tiles of one wave
// (nrect x parts x THETA_TILE^2 doubles at most).
constexpr int CD_MAX_PARTS = 64;
struct CdScratch {
    double *partial = nullptr;
};

// FP32 copies of the operands the sweeps stream, used in the mixed mode: when
// `on`, the snapshots and the maintained-product updates read (and for U, V
// write) these instead of the FP64 arrays, converting to FP64 in registers;
// the Gauss-Seidel stage still reads FP64 blocks and writes FP64 parameters.
struct SweepF32 {
    bool on = false;
    int64_t ldq = 0;            // row length of the q-column arrays: q rounded up to 4
    int64_t ldx = 0;            // row length of Sxx as streamed (p rounded up to 4, or
                                // the slab width in the block-wise mode; padding zero)
    const float *SP = nullptr, *Psi = nullptr, *Sigma = nullptr, *Sxx = nullptr;  // q or p rows
    float *U = nullptr, *V = nullptr;
    int full_rects = -1;        // 64 x 64 rects of the current wave (-1: not known),
                                // set in either precision
};
inline int64_t f32_ld(int64_t cols) { return (cols + 3) / 4 * 4; }

// Activity of every rect of a sweep (1 when the rect holds a coordinate with
// |G| > lambda or a nonzero parameter), decided once at the start of the sweep.
void theta_activity(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t q,
                    const double *GT, const double *Theta, double lamT, int *active);
void lambda_activity(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t q,
                     const double *GL, const double *Lam, double lamL, int *active);

// One wave of the Theta sweep: every rect in `rects` (row- and column-disjoint)
// runs exact Gauss-Seidel over its active coordinates from a snapshot of
// b = 2 Sxy + 2 Sxx V, writes the updated Theta and its delta (dT, nrect
// tiles of THETA_TILE^2), then V[rows, :] += dTheta Sigma[cols, :].
// Sxx: element (k, i) at Sxx[k * ldx + i] for every row k and every column i
// of the wave's tile rows (the full matrix with ldx = p, or a column slab).
void theta_wave(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                int64_t p, int64_t q, const double *Sxx, int64_t ldx, const double *Sxy,
                const double *Sigma, double *V, const double *GT, double *Theta, double lamT,
                double *dT, int *changed, const CdScratch &scr, const WaveProbe *probe = nullptr,
                const SweepF32 *f32 = nullptr);

// The three stages of a Lambda wave (lambda_wave runs them in order).
// lambda_snapshot returns the number of K parts the Gauss-Seidel stage must be
// given.  Within one wave every snapshot must complete before any update
// starts (the updates write rows of U that every snapshot reads).
// The FP32 overloads take the operand copies of the mixed mode; `esz` is the
// byte size of the streamed operands (for the traffic counters).
int lambda_snapshot(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                    int64_t q, const double *SP, const double *U, const double *Psi,
                    const CdScratch &scr, int full = -1);
int lambda_snapshot(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                    int64_t q, const float *SP, const float *U, const float *Psi, int64_t ld,
                    const CdScratch &scr, int full = -1);
void lambda_gauss_seidel(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                         int S, int64_t q, const double *Sigma, const double *Psi,
                         const double *GL, const double *Lam, double lamL, double *D,
                         double *dD, int *changed, const CdScratch &scr,
                         unsigned long long *counters, int esz = 8);
void lambda_update(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t q,
                   const double *Sigma, const double *dD, const int *changed, double *U);
void lambda_update(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t ld,
                   const float *Sigma, const double *dD, const int *changed, float *U);

// One wave of the Lambda direction sweep over upper-triangle rects with
// pairwise-disjoint index sets: exact Gauss-Seidel inside each rect from a
// snapshot of b = G + SP U + (Psi U)^T, D written (both triangles), then
// U rows of both index sets updated with the rect's delta.
void lambda_wave(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                 int64_t q, const double *Sigma, const double *Psi, const double *SP,
                 const double *GL, const double *Lam, double lamL, double *D, double *U,
                 double *dD, int *changed, const CdScratch &scr, const WaveProbe *probe = nullptr,
                 const SweepF32 *f32 = nullptr);

}  // namespace cggm
