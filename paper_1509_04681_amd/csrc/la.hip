// la.hip -- dense FP64 linear algebra on gfx950 for the CGGM solver:
// MFMA GEMM, blocked Cholesky, blocked triangular solve / SPD inverse,
// elementwise assembly and deterministic two-stage reductions.
#include <math.h>

#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace cggm {

namespace {

// --------------------------------------------------------------- GEMM -------
// C = alpha op(A) op(B) + beta C with 128 x 128 output tiles per workgroup:
// each of the 4 waves owns a 64 x 64 quarter as 4 x 4 MFMA 16x16 blocks
// (64 accumulator doubles per lane), so every operand value read from LDS
// feeds four MFMAs.  The K range is staged through LDS in chunks of 16 with
// two buffers: the next chunk's global loads are in flight while the current
// chunk is multiplied, and one barrier per chunk separates the phases.
constexpr int GT = 128;             // output tile edge
constexpr int GKC = 16;             // K chunk
constexpr int GPAD = 8;             // LDS row padding (doubles)
constexpr int GPER = GT * GKC / BLOCK;   // operand elements per thread per chunk (8)

struct GemmSmem {
    double a[2][GKC][GT + GPAD];    // a[buf][k][m] = op(A)[m0 + m][kc + k]
    double b[2][GKC][GT + GPAD];    // b[buf][k][n] = op(B)[kc + k][n0 + n]
};

template <bool TA, bool TB>
__global__ __launch_bounds__(BLOCK) void gemm_kernel(int64_t M, int64_t N, int64_t K,
                                                     double alpha, const double *A, int64_t lda,
                                                     const double *B, int64_t ldb, double beta,
                                                     double *C, int64_t ldc, int uplo,
                                                     int krange) {
    const int64_t bm = blockIdx.y, bn = blockIdx.x;
    if (uplo == UPLO_LOWER && bn > bm) return;
    __shared__ GemmSmem sm;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int64_t m0 = bm * GT, n0 = bn * GT;
    const int64_t k0 = (krange == KRANGE_FROM_ROW) ? std::min<int64_t>(m0, K) : 0;
    const int64_t k1 = K;
    // Element e = tid + BLOCK * r of a chunk: coordinates chosen so that
    // consecutive threads read consecutive addresses of the stored operand.
    auto a_coord = [&](int e, int &k, int &m) {
        if (TA) { k = e / GT; m = e % GT; }
        else { m = e / GKC; k = e % GKC; }
    };
    auto b_coord = [&](int e, int &k, int &n) {
        if (TB) { n = e / GKC; k = e % GKC; }
        else { k = e / GT; n = e % GT; }
    };
    double ra[GPER], rb[GPER];
    auto load = [&](int64_t kc) {
#pragma unroll
        for (int r = 0; r < GPER; ++r) {
            const int e = tid + BLOCK * r;
            int k, m, n;
            a_coord(e, k, m);
            const int64_t gk = kc + k, gm = m0 + m;
            ra[r] = (gk < k1 && gm < M) ? (TA ? A[gk * lda + gm] : A[gm * lda + gk]) : 0.0;
            b_coord(e, k, n);
            const int64_t gk2 = kc + k, gn = n0 + n;
            rb[r] = (gk2 < k1 && gn < N) ? (TB ? B[gn * ldb + gk2] : B[gk2 * ldb + gn]) : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < GPER; ++r) {
            const int e = tid + BLOCK * r;
            int k, m, n;
            a_coord(e, k, m);
            sm.a[buf][k][m] = ra[r];
            b_coord(e, k, n);
            sm.b[buf][k][n] = rb[r];
        }
    };
    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
    const int col = lane & 15, krow = lane >> 4;
    int buf = 0;
    if (k0 < k1) {
        load(k0);
        store(0);
    }
    __syncthreads();
    for (int64_t kc = k0; kc < k1; kc += GKC) {
        const bool next = kc + GKC < k1;
        if (next) load(kc + GKC);
#pragma unroll
        for (int ks = 0; ks < GKC / 4; ++ks) {
            const int k = ks * 4 + krow;
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = sm.a[buf][k][wm + i * 16 + col];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = sm.b[buf][k][wn + j * 16 + col];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma_f64_16x16x4(av[i], bv[j], acc[i][j]);
        }
        if (next) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm + i * 16 + krow + 4 * r;
                const int64_t cc = n0 + wn + j * 16 + col;
                if (row < M && cc < N) {
                    double *c = C + row * ldc + cc;
                    const double v = alpha * acc[i][j][r];
                    *c = (beta == 0.0) ? v : v + beta * (*c);
                }
            }
}

constexpr int GEMM_TS = 64;

// 64 x 64 output tiles (4 waves x 32 x 32), single LDS buffer: used for the
// thin products of the blocked factorizations (K or an output side of 64).
template <bool TA, bool TB>
__global__ __launch_bounds__(BLOCK) void gemm64_kernel(int64_t M, int64_t N, int64_t K,
                                                       double alpha, const double *A,
                                                       int64_t lda, const double *B, int64_t ldb,
                                                       double beta, double *C, int64_t ldc,
                                                       int uplo, int krange) {
    const int64_t bm = blockIdx.y, bn = blockIdx.x;
    if (uplo == UPLO_LOWER && bn > bm) return;
    __shared__ TileSmem<GEMM_TS> sm;
    WaveAcc<GEMM_TS> acc;
    acc.zero();
    const int64_t m0 = bm * GEMM_TS, n0 = bn * GEMM_TS;
    const int64_t k0 = (krange == KRANGE_FROM_ROW) ? std::min<int64_t>(m0, K) : 0;
    tile_mma<TA, TB, GEMM_TS>(A, lda, B, ldb, m0, n0, M, N, k0, K, sm, acc);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
#pragma unroll
    for (int i = 0; i < WaveAcc<GEMM_TS>::NB; ++i)
#pragma unroll
        for (int j = 0; j < WaveAcc<GEMM_TS>::NB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + acc_row<GEMM_TS>(wid, lane, i, r);
                const int64_t col = n0 + acc_col<GEMM_TS>(wid, lane, j);
                if (row < M && col < N) {
                    double *c = C + row * ldc + col;
                    const double v = alpha * acc.c[i][j][r];
                    *c = (beta == 0.0) ? v : v + beta * (*c);
                }
            }
}

// ------------------------------------------------------------ Cholesky ------

// Factor the diagonal block A[kb:kb+nb, kb:kb+nb] = L_kk L_kk^T in LDS (one
// wavefront), store L_kk in place and L_kk^{-1} in Wk (PB x PB, zero above the
// diagonal and outside nb); *notpd = 1 if a pivot is not positive.
//   Factor: left-looking, column j at a time, lane i computes
//     L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj   (L_jj from lane j);
//   inverse: forward substitution by rows, lane c computes
//     W_ic = (delta_ic - sum_{m<i} L_im W_mc) / L_ii.
// Every step is one dot product per lane (two partial sums); the LDS rows are
// padded so a column read across lanes is conflict-free.
__global__ __launch_bounds__(WAVE) void potrf_diag_kernel(double *A, int64_t q, int64_t kb,
                                                          int nb, int *notpd, double *Wk) {
    __shared__ double d[PB][PB + 1];
    __shared__ double w[PB][PB + 1];
    const int lane = threadIdx.x;
#pragma unroll 8
    for (int i = 0; i < PB; ++i)
        d[i][lane] = (i < nb && lane <= i) ? A[(kb + i) * q + kb + lane] : 0.0;
    __syncthreads();
    bool bad = false;
    const bool row_ok = lane < nb;
    for (int j = 0; j < nb; ++j) {
        double a0 = 0.0, a1 = 0.0;
        int k = 0;
        for (; k + 1 < j; k += 2) {
            a0 += d[lane][k] * d[j][k];
            a1 += d[lane][k + 1] * d[j][k + 1];
        }
        if (k < j) a0 += d[lane][k] * d[j][k];
        const double sv = (row_ok && lane >= j) ? d[lane][j] - (a0 + a1) : 0.0;
        const double pivot = readlane_f64(sv, j);
        const bool good = pivot > 0.0 && isfinite(pivot);
        bad |= !good;
        const double ljj = good ? sqrt(pivot) : 1.0;
        if (lane == j)
            d[j][j] = ljj;
        else if (row_ok && lane > j)
            d[lane][j] = sv / ljj;
        __syncthreads();
    }
    for (int i = 0; i < nb; ++i) {
        double a0 = 0.0, a1 = 0.0;
        int m = 0;
        for (; m + 1 < i; m += 2) {
            a0 += d[i][m] * w[m][lane];
            a1 += d[i][m + 1] * w[m + 1][lane];
        }
        if (m < i) a0 += d[i][m] * w[m][lane];
        const double v = ((lane == i) ? 1.0 : 0.0) - (a0 + a1);
        w[i][lane] = (lane <= i) ? v / d[i][i] : 0.0;
        __syncthreads();
    }
#pragma unroll 8
    for (int i = 0; i < PB; ++i) {
        if (i < nb && lane <= i) A[(kb + i) * q + kb + lane] = d[i][lane];
        Wk[i * PB + lane] = (i < nb && lane <= i && lane < nb) ? w[i][lane] : 0.0;
    }
    if (lane == 0 && bad) *notpd = 1;
}

// ---------------------------------------------------------- elementwise -----
__global__ void symmetrize_kernel(int64_t q, double *A) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q * q) return;
    const int64_t i = e / q, j = e % q;
    if (j > i) A[e] = A[j * q + i];
}

__global__ void identity_kernel(int64_t q, double *A) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q * q) return;
    A[e] = (e / q == e % q) ? 1.0 : 0.0;
}

__global__ void transpose_kernel(int64_t rows, int64_t cols, const double *src, double *dst) {
    __shared__ double t[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) t[k][tx] = src[r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;   // dst row c, column r
        if (r < rows && c < cols) dst[c * rows + r] = t[tx][k];
    }
}

__global__ void assemble_lambda_kernel(int64_t count, const double *Syy, const double *Sigma,
                                       const double *Psi, double *GL, double *SP) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const double s = Sigma[e], p = Psi[e];
    GL[e] = Syy[e] - s - p;
    SP[e] = s + p;
}

__global__ void scale_copy_kernel(int64_t count, double a, const double *x, double *y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) y[e] = a * x[e];
}

__global__ void set_int_kernel(int *dst, int v) { *dst = v; }

__global__ void to_f32_kernel(int64_t rows, int64_t cols, const double *__restrict__ x,
                              int64_t ldx, float *__restrict__ y, int64_t ldy) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * ldy) return;
    const int64_t r = e / ldy, c = e % ldy;
    y[e] = c < cols ? (float)x[r * ldx + c] : 0.f;
}

__global__ void fill_f32_kernel(int64_t count, float v, float *__restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) y[e] = v;
}

// ---------------------------------------------------------- reductions ------
// Block-level sum of NV values; thread 0 of the block gets the totals.
template <int NV>
__device__ void block_sum(double (&v)[NV], double (&out)[NV]) {
    __shared__ double red[BLOCK / WAVE][NV];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double w = wave_sum(v[k]);
        if (lane == 0) red[wid][k] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = 0.0;
            for (int w = 0; w < BLOCK / WAVE; ++w) t += red[w][k];
            out[k] = t;
        }
    }
}

template <int NV, class F>
__global__ __launch_bounds__(BLOCK) void reduce_partials_kernel(int64_t count, F f,
                                                                double *partials) {
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < count; e += stride)
        f(e, acc);
    double tot[NV];
    block_sum<NV>(acc, tot);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[blockIdx.x * NV + k] = tot[k];
}

template <int NV>
__global__ __launch_bounds__(BLOCK) void reduce_final_kernel(int nblocks,
                                                             const double *partials,
                                                             double *out) {
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += BLOCK)
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += partials[b * NV + k];
    double tot[NV];
    block_sum<NV>(acc, tot);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = tot[k];
}

template <int NV, class F>
void run_reduce(hipStream_t s, int64_t count, F f, double *partials, double *out) {
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(REDUCE_BLOCKS,
                                                               (count + BLOCK - 1) / BLOCK));
    reduce_partials_kernel<NV, F><<<nb, BLOCK, 0, s>>>(count, f, partials);
    CGGM_LAUNCH_CHECK();
    reduce_final_kernel<NV><<<1, BLOCK, 0, s>>>(nb, partials, out);
    CGGM_LAUNCH_CHECK();
}

struct LogdetF {
    const double *L;
    int64_t q;
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double d = L[i * q + i];
        if (d > 0.0 && isfinite(d)) acc[0] += 2.0 * log(d);
        else acc[1] += 1.0;
    }
};

struct DotF {
    const double *A, *B;
    __device__ void operator()(int64_t e, double (&acc)[1]) const { acc[0] += A[e] * B[e]; }
};

struct TopStatsF {
    const double *W, *G, *P;
    double lam;
    int64_t cols;
    int upper;
    __device__ void operator()(int64_t e, double (&acc)[5]) const {
        const double w = W[e], g = G[e], x = P[e];
        acc[0] += w * x;
        acc[1] += fabs(x);
        if (x != 0.0) acc[2] += fabs(g + copysign(lam, x));
        else acc[2] += fmax(fabs(g) - lam, 0.0);
        const bool in_tri = !upper || (e % cols) >= (e / cols);
        acc[3] += (in_tri && (fabs(g) > lam || x != 0.0)) ? 1.0 : 0.0;
        acc[4] += (x != 0.0) ? 1.0 : 0.0;
    }
};

struct DirectionF {
    const double *G, *Lam, *D;
    __device__ void operator()(int64_t e, double (&acc)[2]) const {
        const double d = D[e], l = Lam[e];
        acc[0] += G[e] * d;
        acc[1] += fabs(l + d) - fabs(l);
    }
};

struct TrialF {
    const double *Lam, *D, *Syy;
    double alpha;
    double *T;
    __device__ void operator()(int64_t e, double (&acc)[2]) const {
        const double t = Lam[e] + alpha * D[e];
        T[e] = t;
        acc[0] += Syy[e] * t;
        acc[1] += fabs(t);
    }
};

struct NonFiniteF {
    const double *x;
    __device__ void operator()(int64_t e, double (&acc)[1]) const {
        acc[0] += isfinite(x[e]) ? 0.0 : 1.0;
    }
};

inline int blocks_for(int64_t count, int bs = BLOCK) {
    return (int)std::max<int64_t>(1, (count + bs - 1) / bs);
}

}  // namespace

// ======================================================== host wrappers =====
void gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
          int64_t ldc, int uplo, int krange) {
    if (M <= 0 || N <= 0) return;
    // Large products take the 128 x 128 tiles; the thin ones of the blocked
    // factorizations (K = 64, or 64 output rows / columns) keep 64 x 64 tiles.
    const bool big = M >= 2 * GT && N >= 2 * GT && K >= 2 * GT;
    const int64_t ts = big ? GT : GEMM_TS;
    dim3 grid((unsigned)((N + ts - 1) / ts), (unsigned)((M + ts - 1) / ts));
#define CGGM_GEMM_LAUNCH(KER)                                                                   \
    do {                                                                                        \
        if (ta && tb)                                                                           \
            KER<true, true><<<grid, BLOCK, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, \
                                                   uplo, krange);                               \
        else if (ta)                                                                            \
            KER<true, false><<<grid, BLOCK, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,     \
                                                    ldc, uplo, krange);                         \
        else if (tb)                                                                            \
            KER<false, true><<<grid, BLOCK, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,     \
                                                    ldc, uplo, krange);                         \
        else                                                                                    \
            KER<false, false><<<grid, BLOCK, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,    \
                                                     ldc, uplo, krange);                        \
    } while (0)
    if (big)
        CGGM_GEMM_LAUNCH(gemm_kernel);
    else
        CGGM_GEMM_LAUNCH(gemm64_kernel);
#undef CGGM_GEMM_LAUNCH
    CGGM_LAUNCH_CHECK();
}

void symmetrize_from_lower(hipStream_t s, int64_t q, double *A) {
    symmetrize_kernel<<<blocks_for(q * q), BLOCK, 0, s>>>(q, A);
    CGGM_LAUNCH_CHECK();
}

void set_identity(hipStream_t s, int64_t q, double *A) {
    identity_kernel<<<blocks_for(q * q), BLOCK, 0, s>>>(q, A);
    CGGM_LAUNCH_CHECK();
}

void transpose(hipStream_t s, int64_t rows, int64_t cols, const double *src, double *dst) {
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    transpose_kernel<<<grid, BLOCK, 0, s>>>(rows, cols, src, dst);
    CGGM_LAUNCH_CHECK();
}

// Outer panel width of the blocked factorizations: a panel of OB columns is
// factored (or solved) with PB-wide steps whose updates stay inside the panel,
// then the rest of the matrix gets one update with K = OB (a large GEMM on the
// 128 x 128 tiles instead of OB / PB thin ones).
constexpr int OB = 4 * PB;

void cholesky_inplace(hipStream_t s, int64_t q, double *A, int *notpd_dev, double *Wd) {
    for (int64_t ob = 0; ob < q; ob += OB) {
        const int64_t oe = std::min<int64_t>(q, ob + OB);
        for (int64_t kb = ob; kb < oe; kb += PB) {
            const int nb = (int)std::min<int64_t>(PB, q - kb);
            const int64_t below = q - kb - nb;
            double *Wk = Wd + (kb / PB) * PB * PB;
            potrf_diag_kernel<<<1, WAVE, 0, s>>>(A, q, kb, nb, notpd_dev, Wk);
            CGGM_LAUNCH_CHECK();
            if (below > 0) {                 // below > 0 implies nb == PB
                // panel: L[below, k] = A[below, k] L_kk^{-T}, in place (one column tile)
                double *Pw = A + (kb + nb) * q + kb;
                gemm(s, false, true, below, nb, nb, 1.0, Pw, q, Wk, PB, 0.0, Pw, q);
                // update of the outer panel's remaining columns [kb + nb, oe)
                const int64_t ncols = oe - (kb + nb);
                if (ncols > 0)
                    gemm(s, false, true, below, ncols, nb, -1.0, Pw, q, Pw, q, 1.0,
                         A + (kb + nb) * q + kb + nb, q, UPLO_LOWER, KRANGE_FULL);
            }
        }
        const int64_t rest = q - oe;
        if (rest > 0) {
            // trailing update with the whole outer panel: A[oe:, oe:] -= P P^T
            const double *P = A + oe * q + ob;
            gemm(s, false, true, rest, rest, oe - ob, -1.0, P, q, P, q, 1.0, A + oe * q + oe, q,
                 UPLO_LOWER, KRANGE_FULL);
        }
    }
}

void trsm_lower_left(hipStream_t s, int64_t q, const double *L, const double *Wd, double *B,
                     int64_t m, int64_t ldb, bool lower_rhs) {
    for (int64_t ob = 0; ob < q; ob += OB) {
        const int64_t oe = std::min<int64_t>(q, ob + OB);
        for (int64_t kb = ob; kb < oe; kb += PB) {
            const int nb = (int)std::min<int64_t>(PB, q - kb);
            const int64_t ncols = lower_rhs ? std::min<int64_t>(m, kb + nb) : m;
            // B_k <- L_kk^{-1} B_k in place (one row tile: every output tile reads its
            // whole K range before it is written)
            gemm(s, false, false, nb, ncols, nb, 1.0, Wd + (kb / PB) * PB * PB, PB,
                 B + kb * ldb, ldb, 0.0, B + kb * ldb, ldb);
            // rows of the outer panel below this block
            const int64_t rows = oe - kb - nb;
            if (rows > 0)
                gemm(s, false, false, rows, ncols, nb, -1.0, L + (kb + nb) * q + kb, q,
                     B + kb * ldb, ldb, 1.0, B + (kb + nb) * ldb, ldb);
        }
        const int64_t rest = q - oe;
        if (rest > 0) {
            // every row below the outer panel: B[oe:] -= L[oe:, ob:oe] B[ob:oe]
            const int64_t ncols = lower_rhs ? std::min<int64_t>(m, oe) : m;
            gemm(s, false, false, rest, ncols, oe - ob, -1.0, L + oe * q + ob, q, B + ob * ldb,
                 ldb, 1.0, B + oe * ldb, ldb);
        }
    }
}

void spd_inverse_from_cholesky(hipStream_t s, int64_t q, const double *L, const double *Wd,
                               double *work, double *Sigma) {
    set_identity(s, q, work);
    trsm_lower_left(s, q, L, Wd, work, q, q, true);      // work = L^{-1} (lower)
    gemm(s, true, false, q, q, q, 1.0, work, q, work, q, 0.0, Sigma, q, UPLO_LOWER,
         KRANGE_FROM_ROW);                               // Sigma = L^{-T} L^{-1}
    symmetrize_from_lower(s, q, Sigma);
}

void reduce_logdet(hipStream_t s, int64_t q, const double *L, double *partials, double *out) {
    run_reduce<2>(s, q, LogdetF{L, q}, partials, out);
}

void reduce_dot(hipStream_t s, int64_t count, const double *A, const double *B,
                double *partials, double *out) {
    run_reduce<1>(s, count, DotF{A, B}, partials, out);
}

void reduce_top_stats(hipStream_t s, int64_t rows, int64_t cols, const double *W,
                      const double *G, const double *P, double lam, int upper,
                      double *partials, double *out) {
    run_reduce<5>(s, rows * cols, TopStatsF{W, G, P, lam, cols, upper}, partials, out);
}

void reduce_direction(hipStream_t s, int64_t q, const double *G, const double *Lam,
                      const double *D, double *partials, double *out) {
    run_reduce<2>(s, q * q, DirectionF{G, Lam, D}, partials, out);
}

void build_trial(hipStream_t s, int64_t q, const double *Lam, const double *D, double alpha,
                 const double *Syy, double *trial, double *partials, double *out) {
    run_reduce<2>(s, q * q, TrialF{Lam, D, Syy, alpha, trial}, partials, out);
}

void reduce_nonfinite(hipStream_t s, int64_t count, const double *x, double *partials,
                      double *out) {
    run_reduce<1>(s, count, NonFiniteF{x}, partials, out);
}

void assemble_lambda_gradient(hipStream_t s, int64_t q, const double *Syy,
                              const double *Sigma, const double *Psi, double *GL, double *SP) {
    assemble_lambda_kernel<<<blocks_for(q * q), BLOCK, 0, s>>>(q * q, Syy, Sigma, Psi, GL, SP);
    CGGM_LAUNCH_CHECK();
}

void scale_copy(hipStream_t s, int64_t count, double a, const double *x, double *y) {
    scale_copy_kernel<<<blocks_for(count), BLOCK, 0, s>>>(count, a, x, y);
    CGGM_LAUNCH_CHECK();
}

void to_f32(hipStream_t s, int64_t rows, int64_t cols, const double *x, int64_t ldx, float *y,
            int64_t ldy) {
    const int64_t count = rows * ldy;
    if (count <= 0) return;
    to_f32_kernel<<<(unsigned)((count + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(rows, cols, x, ldx, y,
                                                                            ldy);
    CGGM_LAUNCH_CHECK();
}

void fill_f32(hipStream_t s, int64_t count, float v, float *y) {
    if (count <= 0) return;
    fill_f32_kernel<<<(unsigned)((count + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(count, v, y);
    CGGM_LAUNCH_CHECK();
}

void set_int(hipStream_t s, int *dst, int v) {
    set_int_kernel<<<1, 1, 0, s>>>(dst, v);
    CGGM_LAUNCH_CHECK();
}

}  // namespace cggm
