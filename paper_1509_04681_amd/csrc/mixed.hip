// mixed.hip -- split-BF16 products with FP32 accumulation on gfx950 (the
// mixed-precision mode of the solver).
//
// An FP64 value x is split into three BF16 values hi + mid + lo: hi = bf16(x),
// mid = bf16(x - hi), lo = bf16(x - hi - mid); the residuals are exact in FP64,
// so x - (hi + mid + lo) is below 2^-24 |x| or so.  A product sum
// sum_k a_k b_k is then formed from the six cross products whose pieces carry
// most of the value -- hi*hi, hi*mid, mid*hi, mid*mid, hi*lo, lo*hi -- on the
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32 accumulation.  The
// result differs from the FP64 product by about the FP32 accumulation error
// (a few 1e-6 relative over tens of thousands of terms).
#include <math.h>

#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace cggm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// planes[t][r * ldp + c] for t = 0, 1, 2 (hi, mid, lo), c < cols; zero for
// cols <= c < ldp.
__global__ void split3_kernel(const double *__restrict__ X, int64_t rows, int64_t cols,
                              int64_t ldx, int64_t ldp, __bf16 *__restrict__ planes) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * ldp) return;
    const int64_t r = e / ldp, c = e % ldp;
    const double x = c < cols ? X[r * ldx + c] : 0.0;
    const __bf16 hi = (__bf16)(float)x;
    const double r1 = x - (double)(float)hi;
    const __bf16 mid = (__bf16)(float)r1;
    const double r2 = r1 - (double)(float)mid;
    const __bf16 lo = (__bf16)(float)r2;
    const int64_t plane = rows * ldp;
    planes[e] = hi;
    planes[plane + e] = mid;
    planes[2 * plane + e] = lo;
}

constexpr int MT = 128;          // output tile edge
constexpr int MK = 32;           // K per MFMA step
constexpr int MPAD = 8;          // LDS row padding (bf16)
constexpr int MROW = MK + MPAD;  // LDS row length (bf16), 80 bytes
constexpr int MLOADS = 3 * MT * MK / 8 / BLOCK;   // 16-byte loads per thread per operand (6)

struct MixSmem {
    __bf16 a[3][MT][MROW];    // a[plane][m][k] of the current K step
    __bf16 b[3][MT][MROW];    // b[plane][n][k]
};

// C (M x N, FP64) = A B^T from the split planes of A (M x Kp, row length Kp)
// and B (N x Kp): 128 x 128 tiles, each of the 4 waves a 64 x 64 quarter as
// 4 x 4 MFMA blocks with FP32 accumulators.  The next K step's planes are
// loaded into registers while the current one is multiplied from LDS.
template <class TC>
__global__ __launch_bounds__(BLOCK) void gemm_split3_nt_kernel(int64_t M, int64_t N, int64_t Kp,
                                                               const __bf16 *__restrict__ Ap,
                                                               const __bf16 *__restrict__ Bp,
                                                               TC *__restrict__ C, int64_t ldc) {
    __shared__ MixSmem sm;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int64_t m0 = (int64_t)blockIdx.y * MT, n0 = (int64_t)blockIdx.x * MT;
    const int64_t aplane = M * Kp, bplane = N * Kp;
    uint4 ra[MLOADS], rb[MLOADS];
    // element e = tid + BLOCK * r: plane e / 512, row (e % 512) / 4, 8-wide
    // k chunk e % 4 -- consecutive threads read consecutive 16-byte pieces
#define MIX_LOAD(KC)                                                                      \
    _Pragma("unroll") for (int r = 0; r < MLOADS; ++r) {                                  \
        const int e = tid + BLOCK * r;                                                    \
        const int pl = e / (MT * 4), row = (e % (MT * 4)) / 4, ch = e % 4;                \
        const int64_t gm = m0 + row, gn = n0 + row;                                       \
        /* rows past the matrix read its last row and are replaced by zeros */            \
        const uint4 va = *reinterpret_cast<const uint4 *>(                                \
            Ap + pl * aplane + std::min<int64_t>(gm, M - 1) * Kp + (KC) + ch * 8);        \
        const uint4 vb = *reinterpret_cast<const uint4 *>(                                \
            Bp + pl * bplane + std::min<int64_t>(gn, N - 1) * Kp + (KC) + ch * 8);        \
        const bool oka = gm < M, okb = gn < N;                                            \
        ra[r] = uint4{oka ? va.x : 0u, oka ? va.y : 0u, oka ? va.z : 0u, oka ? va.w : 0u}; \
        rb[r] = uint4{okb ? vb.x : 0u, okb ? vb.y : 0u, okb ? vb.z : 0u, okb ? vb.w : 0u}; \
    }
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
    const int col = lane & 15, kq = (lane >> 4) * 8;
    MIX_LOAD(0)
    for (int64_t kc = 0; kc < Kp; kc += MK) {
        __syncthreads();                      // the previous step's reads are done
#pragma unroll
        for (int r = 0; r < MLOADS; ++r) {
            const int e = tid + BLOCK * r;
            const int pl = e / (MT * 4), row = (e % (MT * 4)) / 4, ch = e % 4;
            *reinterpret_cast<uint4 *>(&sm.a[pl][row][ch * 8]) = ra[r];
            *reinterpret_cast<uint4 *>(&sm.b[pl][row][ch * 8]) = rb[r];
        }
        __syncthreads();
        if (kc + MK < Kp) {
            MIX_LOAD(kc + MK)
        }
        uint4 bu[3][4];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bu[p][j] = *reinterpret_cast<const uint4 *>(&sm.b[p][wn + j * 16 + col][kq]);
#pragma unroll
        for (int pa = 0; pa < 3; ++pa) {
            uint4 au[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                au[i] = *reinterpret_cast<const uint4 *>(&sm.a[pa][wm + i * 16 + col][kq]);
            // piece pa of A against the pieces pb of B with pa + pb <= 2
#pragma unroll
            for (int pb = 0; pb < 3; ++pb) {
                if (pa + pb > 2) continue;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, au[i]), __builtin_bit_cast(bf16x8, bu[pb][j]),
                            acc[i][j], 0, 0, 0);
            }
        }
    }
#undef MIX_LOAD
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int64_t cc = n0 + wn + j * 16 + col;
                if (row < M && cc < N) C[row * ldc + cc] = (TC)acc[i][j][r];
            }
}

}  // namespace

int64_t split3_stride(int64_t K) { return (K + MK - 1) / MK * MK; }

void split3(hipStream_t s, int64_t rows, int64_t cols, const double *X, int64_t ldx,
            __bf16 *planes) {
    const int64_t ldp = split3_stride(cols);
    const int64_t count = rows * ldp;
    if (count <= 0) return;
    split3_kernel<<<(unsigned)((count + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(X, rows, cols, ldx,
                                                                           ldp, planes);
    CGGM_LAUNCH_CHECK();
}

template <class TC>
void gemm_split3_nt_t(hipStream_t s, int64_t M, int64_t N, int64_t K, const __bf16 *Ap,
                      const __bf16 *Bp, TC *C, int64_t ldc) {
    if (M <= 0 || N <= 0) return;
    dim3 grid((unsigned)((N + MT - 1) / MT), (unsigned)((M + MT - 1) / MT));
    gemm_split3_nt_kernel<TC><<<grid, BLOCK, 0, s>>>(M, N, split3_stride(K), Ap, Bp, C, ldc);
    CGGM_LAUNCH_CHECK();
}

void gemm_split3_nt(hipStream_t s, int64_t M, int64_t N, int64_t K, const __bf16 *Ap,
                    const __bf16 *Bp, double *C, int64_t ldc) {
    gemm_split3_nt_t<double>(s, M, N, K, Ap, Bp, C, ldc);
}

void gemm_split3_nt(hipStream_t s, int64_t M, int64_t N, int64_t K, const __bf16 *Ap,
                    const __bf16 *Bp, float *C, int64_t ldc) {
    gemm_split3_nt_t<float>(s, M, N, K, Ap, Bp, C, ldc);
}

}  // namespace cggm
