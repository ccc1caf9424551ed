// cg.hip -- columns of Sigma = Lambda^{-1} by conjugate gradients on a sparse
// symmetric positive definite Lambda, the way the block-wise method of
// Sec. 4.1 obtains the Sigma columns a block needs without a dense
// factorization: O(m_Lambda) work per iteration and column.  The columns of a
// batch (up to 64, one per lane) advance together, so each iteration is one
// sparse-by-dense product Lambda P (q x 64) and a few streaming updates; every
// reduction is a fixed-order sum over fixed partials (deterministic).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "cggm.h"
#include "device_common.hpp"
#include "internal.hpp"
#include "solver.hpp"

namespace cggm {
namespace {

constexpr int CG_COLS = 64;                          // columns per batch: one per lane
constexpr int CG_BLOCKS = 1024;                      // workgroups of the row kernels
constexpr int CG_WAVES = CG_BLOCKS * (BLOCK / WAVE); // waves of the row kernels
constexpr int CG_CHECK = 8;                          // iterations between host checks

// flag[0]: a CSR column index outside [0, q); flag[1]: a column met a
// curvature p^T Lambda p that is not positive.
enum { FLAG_BADCOL = 0, FLAG_NOTPD = 1 };

__global__ __launch_bounds__(BLOCK) void cg_check_cols_kernel(const int32_t *__restrict__ col,
                                                              int64_t nnz, int64_t q,
                                                              int *__restrict__ flag) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * BLOCK) {
        const int32_t j = col[t];
        if (j < 0 || j >= q) flag[FLAG_BADCOL] = 1;
    }
}

// X = 0, R = P = E (column c of the batch is e_{cols[c]}), rr = 1 for the
// batch's columns; padding columns (c >= kb) start converged.
__global__ __launch_bounds__(BLOCK) void cg_init_kernel(int64_t q, const int32_t *__restrict__ cols,
                                                        int kb, double *__restrict__ X,
                                                        double *__restrict__ R,
                                                        double *__restrict__ P,
                                                        double *__restrict__ rr,
                                                        int *__restrict__ done,
                                                        int *__restrict__ flag) {
    const int64_t total = q * CG_COLS;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * BLOCK) {
        const int64_t i = e / CG_COLS;
        const int c = (int)(e % CG_COLS);
        const double v = (c < kb && cols[c] == i) ? 1.0 : 0.0;
        X[e] = 0.0;
        R[e] = v;
        P[e] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x < CG_COLS) {
        const int c = threadIdx.x;
        rr[c] = c < kb ? 1.0 : 0.0;
        done[c] = c < kb ? 0 : 1;
        if (c == 0) flag[FLAG_NOTPD] = 0;
    }
}

// AP = Lambda P, one wave per row (lane = column), and per-wave partial
// sums of P .* AP per column into part[wave][c].
__global__ __launch_bounds__(BLOCK) void cg_spmv_kernel(int64_t q, const int64_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ P,
                                                        double *__restrict__ AP,
                                                        double *__restrict__ part) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t gw = (int64_t)blockIdx.x * (BLOCK / WAVE) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    double dot = 0.0;
    for (int64_t i = gw; i < q; i += CG_WAVES) {
        const int64_t b = rowptr[i], e = rowptr[i + 1];
        double s0 = 0.0, s1 = 0.0;
        int64_t t = b;
        for (; t + 4 <= e; t += 4) {
            const int64_t j0 = col[t], j1 = col[t + 1], j2 = col[t + 2], j3 = col[t + 3];
            const double v0 = val[t], v1 = val[t + 1], v2 = val[t + 2], v3 = val[t + 3];
            const double p0 = P[j0 * CG_COLS + lane], p1 = P[j1 * CG_COLS + lane];
            const double p2 = P[j2 * CG_COLS + lane], p3 = P[j3 * CG_COLS + lane];
            s0 = fma(v0, p0, s0);
            s1 = fma(v1, p1, s1);
            s0 = fma(v2, p2, s0);
            s1 = fma(v3, p3, s1);
        }
        for (; t < e; ++t) s0 = fma(val[t], P[(int64_t)col[t] * CG_COLS + lane], s0);
        const double s = s0 + s1;
        AP[i * CG_COLS + lane] = s;
        dot = fma(P[i * CG_COLS + lane], s, dot);
    }
    part[gw * CG_COLS + lane] = dot;
}

// out[c] = sum over the waves of part[w][c], in wave order per thread and a
// fixed tree over the threads: one workgroup per column.
__global__ __launch_bounds__(BLOCK) void cg_reduce_kernel(const double *__restrict__ part,
                                                          double *__restrict__ out) {
    __shared__ double red[BLOCK];
    const int c = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int w = tid; w < CG_WAVES; w += BLOCK) s += part[(int64_t)w * CG_COLS + c];
    red[tid] = s;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) out[c] = red[0];
}

// alpha = rr / pAp per column (zero for converged columns and for a
// curvature that is not positive); X += alpha P, R -= alpha AP, and per-wave
// partial sums of R .* R.
__global__ __launch_bounds__(BLOCK) void cg_axpy_kernel(int64_t q, double *__restrict__ X,
                                                        double *__restrict__ R,
                                                        const double *__restrict__ P,
                                                        const double *__restrict__ AP,
                                                        const double *__restrict__ rr,
                                                        const double *__restrict__ pap,
                                                        const int *__restrict__ done,
                                                        double *__restrict__ part) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t gw = (int64_t)blockIdx.x * (BLOCK / WAVE) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const double den = pap[lane];
    const double alpha = (!done[lane] && den > 0.0) ? rr[lane] / den : 0.0;
    double dot = 0.0;
    for (int64_t i = gw; i < q; i += CG_WAVES) {
        const int64_t o = i * CG_COLS + lane;
        double r = R[o];
        if (alpha != 0.0) {
            X[o] = fma(alpha, P[o], X[o]);
            r = fma(-alpha, AP[o], r);
            R[o] = r;
        }
        dot = fma(r, r, dot);
    }
    part[gw * CG_COLS + lane] = dot;
}

// P = R + beta P with beta = rr_new / rr, for the columns not yet converged.
__global__ __launch_bounds__(BLOCK) void cg_direction_kernel(int64_t q, const double *__restrict__ R,
                                                             double *__restrict__ P,
                                                             const double *__restrict__ rr,
                                                             const double *__restrict__ rr_new,
                                                             const int *__restrict__ done) {
    const int64_t total = q * CG_COLS;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * BLOCK) {
        const int c = (int)(e % CG_COLS);
        if (done[c]) continue;
        const double beta = rr[c] > 0.0 ? rr_new[c] / rr[c] : 0.0;
        P[e] = fma(beta, P[e], R[e]);
    }
}

// Per column: flag a curvature that is not positive, take rr = rr_new and
// mark the column converged once its residual norm is at most tol.
__global__ void cg_scalar_kernel(double *__restrict__ rr, const double *__restrict__ rr_new,
                                 const double *__restrict__ pap, int *__restrict__ done,
                                 int *__restrict__ flag, double tol) {
    const int c = threadIdx.x;
    if (c >= CG_COLS || done[c]) return;
    if (!(pap[c] > 0.0)) flag[FLAG_NOTPD] = 1;
    rr[c] = rr_new[c];
    if (sqrt(rr_new[c]) <= tol) done[c] = 1;
}

// out[i * ldo + c] = X[i][c] for the kb columns of the batch.
__global__ __launch_bounds__(BLOCK) void cg_store_kernel(int64_t q, int kb,
                                                         const double *__restrict__ X,
                                                         double *__restrict__ out, int64_t ldo) {
    const int64_t total = q * CG_COLS;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * BLOCK) {
        const int64_t i = e / CG_COLS;
        const int c = (int)(e % CG_COLS);
        if (c < kb) out[i * ldo + c] = X[e];
    }
}

unsigned stream_blocks(int64_t elems) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((elems + BLOCK - 1) / BLOCK, 4096));
}

// Device memory of one call, freed on every exit path.
struct DevBuf {
    void *p = nullptr;
    explicit DevBuf(size_t bytes) {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(CGGM_ENOMEM, "conjugate-gradient workspace of " + std::to_string(bytes) +
                                  " bytes");
        }
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

int sigma_columns_impl(const int64_t *rowptr, const int32_t *col, const double *val, int64_t q,
                       const int32_t *cols, int64_t k, double tol, int max_iter, double *out,
                       int *iters_out, double *resid_out, hipStream_t s) {
    if (q < 1 || k < 0 || max_iter < 1 || !(tol >= 0.0) || !std::isfinite(tol))
        fail(CGGM_EINVAL, "sigma_columns: q >= 1, k >= 0, max_iter >= 1 and a finite tol >= 0 "
                          "are required");
    if (k > 0 && (!rowptr || !col || !val || !cols || !out))
        fail(CGGM_EINVAL, "sigma_columns: null pointer");
    for (int64_t t = 0; t < k; ++t)
        if (cols[t] < 0 || cols[t] >= q)
            fail(CGGM_EINVAL, "sigma_columns: column index " + std::to_string(cols[t]) +
                                  " outside [0, q)");
    if (iters_out) *iters_out = 0;
    if (resid_out) *resid_out = 0.0;
    if (k == 0) return CGGM_OK;

    // the row pointers bound every access of the product: check them on the host
    std::vector<int64_t> rp(q + 1);
    CGGM_HIP(hipMemcpyAsync(rp.data(), rowptr, sizeof(int64_t) * (q + 1), hipMemcpyDeviceToHost,
                            s));
    CGGM_HIP(hipStreamSynchronize(s));
    if (rp[0] != 0) fail(CGGM_EINVAL, "sigma_columns: rowptr[0] != 0");
    for (int64_t i = 0; i < q; ++i)
        if (rp[i + 1] < rp[i]) fail(CGGM_EINVAL, "sigma_columns: rowptr decreases");
    const int64_t nnz = rp[q];

    const size_t zb = sizeof(double) * (size_t)q * CG_COLS;
    const size_t partb = sizeof(double) * (size_t)CG_WAVES * CG_COLS;
    DevBuf buf(4 * zb + partb + 3 * CG_COLS * sizeof(double) +
               (CG_COLS + 2 + CG_COLS) * sizeof(int));
    char *base = static_cast<char *>(buf.p);
    double *X = reinterpret_cast<double *>(base);
    double *R = reinterpret_cast<double *>(base + zb);
    double *P = reinterpret_cast<double *>(base + 2 * zb);
    double *AP = reinterpret_cast<double *>(base + 3 * zb);
    double *part = reinterpret_cast<double *>(base + 4 * zb);
    double *rr = part + (size_t)CG_WAVES * CG_COLS;
    double *rr_new = rr + CG_COLS;
    double *pap = rr_new + CG_COLS;
    int *done = reinterpret_cast<int *>(pap + CG_COLS);
    int *flag = done + CG_COLS;
    int32_t *cols_dev = flag + 2;

    int hflag[2] = {0, 0};
    CGGM_HIP(hipMemcpyAsync(flag, hflag, sizeof(hflag), hipMemcpyHostToDevice, s));
    if (nnz > 0) {
        cg_check_cols_kernel<<<stream_blocks(nnz), BLOCK, 0, s>>>(col, nnz, q, flag);
        CGGM_LAUNCH_CHECK();
    }
    CGGM_HIP(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
    CGGM_HIP(hipStreamSynchronize(s));
    if (hflag[FLAG_BADCOL]) fail(CGGM_EINVAL, "sigma_columns: CSR column index outside [0, q)");

    const unsigned zblocks = stream_blocks(q * CG_COLS);
    int iters_max = 0;
    double resid = 0.0;
    bool all_converged = true;
    std::vector<int32_t> hcols(CG_COLS);
    std::vector<int> hdone(CG_COLS);
    std::vector<double> hrr(CG_COLS);
    for (int64_t t0 = 0; t0 < k; t0 += CG_COLS) {
        const int kb = (int)std::min<int64_t>(CG_COLS, k - t0);
        std::fill(hcols.begin(), hcols.end(), -1);
        std::copy(cols + t0, cols + t0 + kb, hcols.begin());
        CGGM_HIP(hipMemcpyAsync(cols_dev, hcols.data(), sizeof(int32_t) * CG_COLS,
                                hipMemcpyHostToDevice, s));
        cg_init_kernel<<<zblocks, BLOCK, 0, s>>>(q, cols_dev, kb, X, R, P, rr, done, flag);
        CGGM_LAUNCH_CHECK();
        int it = 0;
        bool converged = false;
        while (it < max_iter) {
            cg_spmv_kernel<<<CG_BLOCKS, BLOCK, 0, s>>>(q, rowptr, col, val, P, AP, part);
            CGGM_LAUNCH_CHECK();
            cg_reduce_kernel<<<CG_COLS, BLOCK, 0, s>>>(part, pap);
            CGGM_LAUNCH_CHECK();
            cg_axpy_kernel<<<CG_BLOCKS, BLOCK, 0, s>>>(q, X, R, P, AP, rr, pap, done, part);
            CGGM_LAUNCH_CHECK();
            cg_reduce_kernel<<<CG_COLS, BLOCK, 0, s>>>(part, rr_new);
            CGGM_LAUNCH_CHECK();
            cg_direction_kernel<<<zblocks, BLOCK, 0, s>>>(q, R, P, rr, rr_new, done);
            CGGM_LAUNCH_CHECK();
            cg_scalar_kernel<<<1, CG_COLS, 0, s>>>(rr, rr_new, pap, done, flag, tol);
            CGGM_LAUNCH_CHECK();
            ++it;
            if (it % CG_CHECK == 0 || it == max_iter) {
                CGGM_HIP(hipMemcpyAsync(hdone.data(), done, sizeof(int) * CG_COLS,
                                        hipMemcpyDeviceToHost, s));
                CGGM_HIP(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
                CGGM_HIP(hipStreamSynchronize(s));
                if (hflag[FLAG_NOTPD])
                    fail(CGGM_ENOTPD, "sigma_columns: a curvature p^T Lambda p is not positive");
                converged = std::all_of(hdone.begin(), hdone.end(), [](int d) { return d != 0; });
                if (converged) break;
            }
        }
        cg_store_kernel<<<zblocks, BLOCK, 0, s>>>(q, kb, X, out + t0, k);
        CGGM_LAUNCH_CHECK();
        CGGM_HIP(hipMemcpyAsync(hrr.data(), rr, sizeof(double) * CG_COLS, hipMemcpyDeviceToHost,
                                s));
        CGGM_HIP(hipStreamSynchronize(s));
        for (int c = 0; c < kb; ++c) resid = std::max(resid, sqrt(hrr[c]));
        iters_max = std::max(iters_max, it);
        all_converged = all_converged && converged;
    }
    if (iters_out) *iters_out = iters_max;
    if (resid_out) *resid_out = resid;
    return all_converged ? CGGM_OK : CGGM_MAXITER;
}

}  // namespace
}  // namespace cggm

extern "C" int cggm_sigma_columns(const int64_t *rowptr, const int32_t *col, const double *val,
                                  int64_t q, const int32_t *cols, int64_t k, double tol,
                                  int max_iter, double *Sigma_C, int *iters, double *resid,
                                  void *stream) {
    return cggm::guarded([&] {
        return cggm::sigma_columns_impl(rowptr, col, val, q, cols, k, tol, max_iter, Sigma_C,
                                        iters, resid, (hipStream_t)stream);
    });
}
