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
                                                     // (one partial each per column)
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

// X = 0, R = E (column c of the batch is e_{cols[c]}), the previous
// direction P0 = 0 (the first direction is then R), rr = 1 for the batch's
// columns; padding columns (c >= kb) start converged.
__global__ __launch_bounds__(BLOCK) void cg_init_kernel(int64_t q, const int32_t *__restrict__ cols,
                                                        int kb, double *__restrict__ X,
                                                        double *__restrict__ R,
                                                        double *__restrict__ P0,
                                                        double *__restrict__ rr,
                                                        int *__restrict__ done,
                                                        int *__restrict__ flag) {
    const int64_t total = q * CG_COLS;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * BLOCK) {
        const int64_t i = e / CG_COLS;
        const int c = (int)(e % CG_COLS);
        X[e] = 0.0;
        R[e] = (c < kb && cols[c] == i) ? 1.0 : 0.0;
        P0[e] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x < CG_COLS) {
        const int c = threadIdx.x;
        rr[c] = c < kb ? 1.0 : 0.0;
        done[c] = c < kb ? 0 : 1;
        if (c == 0) flag[FLAG_NOTPD] = 0;
    }
}

// The four waves' per-lane values summed in wave order into
// part[block][lane] (one partial per workgroup and column).
__device__ __forceinline__ void block_partial(double v, double *__restrict__ part) {
    __shared__ double red[BLOCK / WAVE][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    red[wid][lane] = v;
    __syncthreads();
    if (wid == 0)
        part[(int64_t)blockIdx.x * CG_COLS + lane] =
            (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Row i of the new direction and of the product: every P entry the row
// reads is formed on the fly as R + beta Pold (bit for bit the value row j
// writes for itself), the entries of the row taken four at a time with the
// index clamped into the row and the value of a missing entry zero.
struct CgRow {
    double ap, p;      // (Lambda Pnew)_i and Pnew_i of this lane's column
};
__device__ __forceinline__ CgRow cg_row(int64_t i, int lane, double beta,
                                        const int64_t *__restrict__ rowptr,
                                        const int32_t *__restrict__ col,
                                        const double *__restrict__ val,
                                        const double *__restrict__ R,
                                        const double *__restrict__ Pold) {
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t t = b; t < e; t += 4) {
        int64_t j[4];
        double v[4], pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t tu = t + u < e ? t + u : e - 1;
            j[u] = col[tu];
            v[u] = t + u < e ? val[tu] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t o = j[u] * CG_COLS + lane;
            pj[u] = fma(beta, Pold[o], R[o]);
        }
        s0 = fma(v[0], pj[0], s0);
        s1 = fma(v[1], pj[1], s1);
        s0 = fma(v[2], pj[2], s0);
        s1 = fma(v[3], pj[3], s1);
    }
    const int64_t o = i * CG_COLS + lane;
    return CgRow{s0 + s1, fma(beta, Pold[o], R[o])};
}

// Pnew = R + beta Pold with beta = rr / rr_prev (0 on the first iteration
// and for converged columns), AP = Lambda Pnew, one wave per row (lane =
// column; two rows of the wave in flight), and per-workgroup partial sums of
// Pnew .* AP per column.
__global__ __launch_bounds__(BLOCK) void cg_product_kernel(
    int64_t q, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ R,
    const double *__restrict__ Pold, double *__restrict__ Pnew, double *__restrict__ AP,
    const double *__restrict__ rr, const double *__restrict__ rr_prev,
    const int *__restrict__ done, int first, double *__restrict__ part) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t gw = (int64_t)blockIdx.x * (BLOCK / WAVE) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const double beta =
        (first || done[lane] || !(rr_prev[lane] > 0.0)) ? 0.0 : rr[lane] / rr_prev[lane];
    double dot = 0.0;
    for (int64_t i = gw; i < q; i += 2 * CG_WAVES) {
        const int64_t i2 = i + CG_WAVES;
        const CgRow a = cg_row(i, lane, beta, rowptr, col, val, R, Pold);
        if (i2 < q) {
            const CgRow c = cg_row(i2, lane, beta, rowptr, col, val, R, Pold);
            Pnew[i2 * CG_COLS + lane] = c.p;
            AP[i2 * CG_COLS + lane] = c.ap;
            dot = fma(c.p, c.ap, dot);
        }
        Pnew[i * CG_COLS + lane] = a.p;
        AP[i * CG_COLS + lane] = a.ap;
        dot = fma(a.p, a.ap, dot);
    }
    block_partial(dot, part);
}

// out[c] = sum of the CG_BLOCKS partials of column c, in block order per
// thread and a fixed tree over the threads: one workgroup per column.  With
// `tail`, the column's step also ends here: a curvature that is not positive
// is flagged, and the column is marked converged once its residual norm
// sqrt(out[c]) is at most tol.
__global__ __launch_bounds__(BLOCK) void cg_reduce_kernel(const double *__restrict__ part,
                                                          double *__restrict__ out, int tail,
                                                          const double *__restrict__ pap,
                                                          int *__restrict__ done,
                                                          int *__restrict__ flag, double tol) {
    __shared__ double red[BLOCK];
    const int c = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int w = tid; w < CG_BLOCKS; w += BLOCK) s += part[(int64_t)w * CG_COLS + c];
    red[tid] = s;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        out[c] = red[0];
        if (tail && !done[c]) {
            if (!(pap[c] > 0.0)) flag[FLAG_NOTPD] = 1;
            if (sqrt(red[0]) <= tol) done[c] = 1;
        }
    }
}

// alpha = rr / pAp per column (zero for converged columns and for a
// curvature that is not positive); X += alpha P, R -= alpha AP (two rows of
// the wave in flight), and per-workgroup partial sums of R .* R.
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
    for (int64_t i = gw; i < q; i += 2 * CG_WAVES) {
        const int64_t o = i * CG_COLS + lane, o2 = o + (int64_t)CG_WAVES * CG_COLS;
        const bool has2 = i + CG_WAVES < q;
        double r = R[o], r2 = has2 ? R[o2] : 0.0;
        if (alpha != 0.0) {
            const double x = X[o], p = P[o], ap = AP[o];
            double x2 = 0.0, p2 = 0.0, ap2 = 0.0;
            if (has2) {
                x2 = X[o2];
                p2 = P[o2];
                ap2 = AP[o2];
            }
            X[o] = fma(alpha, p, x);
            r = fma(-alpha, ap, r);
            R[o] = r;
            if (has2) {
                X[o2] = fma(alpha, p2, x2);
                r2 = fma(-alpha, ap2, r2);
                R[o2] = r2;
            }
        }
        dot = fma(r, r, dot);
        dot = fma(r2, r2, dot);
    }
    block_partial(dot, part);
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
    const size_t partb = sizeof(double) * (size_t)CG_BLOCKS * CG_COLS;
    DevBuf buf(5 * zb + partb + 3 * CG_COLS * sizeof(double) +
               (CG_COLS + 2 + CG_COLS) * sizeof(int));
    char *base = static_cast<char *>(buf.p);
    double *X = reinterpret_cast<double *>(base);
    double *R = reinterpret_cast<double *>(base + zb);
    double *Pb[2] = {reinterpret_cast<double *>(base + 2 * zb),
                     reinterpret_cast<double *>(base + 3 * zb)};
    double *AP = reinterpret_cast<double *>(base + 4 * zb);
    double *part = reinterpret_cast<double *>(base + 5 * zb);
    double *rrb = part + (size_t)CG_BLOCKS * CG_COLS;   // two slots of CG_COLS
    double *pap = rrb + 2 * CG_COLS;
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
        cg_init_kernel<<<zblocks, BLOCK, 0, s>>>(q, cols_dev, kb, X, R, Pb[0], rrb, done, flag);
        CGGM_LAUNCH_CHECK();
        int it = 0;
        bool converged = false;
        while (it < max_iter) {
            // iteration it: rr in slot it & 1 (the previous one in the other
            // slot, which this iteration's new rr replaces); direction it - 1
            // in Pb[it & 1], the new one into Pb[(it + 1) & 1]
            double *rr = rrb + (it & 1) * CG_COLS, *rr_other = rrb + ((it + 1) & 1) * CG_COLS;
            const double *Pold = Pb[it & 1];
            double *Pnew = Pb[(it + 1) & 1];
            cg_product_kernel<<<CG_BLOCKS, BLOCK, 0, s>>>(q, rowptr, col, val, R, Pold, Pnew, AP,
                                                          rr, rr_other, done, it == 0, part);
            CGGM_LAUNCH_CHECK();
            cg_reduce_kernel<<<CG_COLS, BLOCK, 0, s>>>(part, pap, 0, nullptr, nullptr, nullptr,
                                                       tol);
            CGGM_LAUNCH_CHECK();
            cg_axpy_kernel<<<CG_BLOCKS, BLOCK, 0, s>>>(q, X, R, Pnew, AP, rr, pap, done, part);
            CGGM_LAUNCH_CHECK();
            cg_reduce_kernel<<<CG_COLS, BLOCK, 0, s>>>(part, rr_other, 1, pap, done, flag, tol);
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
        CGGM_HIP(hipMemcpyAsync(hrr.data(), rrb + (it & 1) * CG_COLS, sizeof(double) * CG_COLS,
                                hipMemcpyDeviceToHost, s));
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
