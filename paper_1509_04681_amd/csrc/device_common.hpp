// device_common.hpp -- device-side building blocks shared by the kernels of the
// gfx950 CGGM solver: the FP64 MFMA tile product, wave-level helpers and
// the soft-threshold operator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cggm {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr int BLOCK = 256;      // 4 waves per workgroup
constexpr int KCH = 16;         // K chunk staged through LDS
constexpr int LDS_PAD = 2;      // row padding (doubles) of the staged chunks

// One v_mfma_f64_16x16x4_f64: D(16x16) += A(16x4) B(4x16).
// Operand layout per lane l: A[l % 16][l / 16], B[l / 16][l % 16];
// result element r of lane l is D[l / 16 + 4 * r][l % 16].
__device__ __forceinline__ v4d mfma_f64_16x16x4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS staging buffers of a TS x TS tile product (TS = 32 or 64).
template <int TS>
struct TileSmem {
    double a[KCH][TS + LDS_PAD];   // a[k][m] = op(A)[m0 + m][kc + k]
    double b[KCH][TS + LDS_PAD];   // b[k][n] = op(B)[kc + k][n0 + n]
};

// Accumulator of one wave: its (TS/2) x (TS/2) quadrant of the tile as
// NB x NB MFMA 16x16 blocks (NB = TS / 32).  Wave w owns rows (w >> 1) * TS/2
// and columns (w & 1) * TS/2.
template <int TS>
struct WaveAcc {
    static constexpr int NB = TS / 32;
    v4d c[NB][NB];
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) c[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
};

// Row / column inside the TS x TS tile of accumulator element (i, j, r) of
// `lane` in wave `wid`.
template <int TS>
__device__ __forceinline__ int acc_row(int wid, int lane, int i, int r) {
    return (wid >> 1) * (TS / 2) + i * 16 + (lane >> 4) + 4 * r;
}
template <int TS>
__device__ __forceinline__ int acc_col(int wid, int lane, int j) {
    return (wid & 1) * (TS / 2) + j * 16 + (lane & 15);
}

// acc += op(A)[m0:m0+TS, k0:k1] * op(B)[k0:k1, n0:n0+TS] for one TS x TS tile,
// with rows >= M and columns >= N read as zero.
//   op(A)[m][k] = TA ? A[k * lda + m] : A[m * lda + k]
//   op(B)[k][n] = TB ? B[n * ldb + k] : B[k * ldb + n]
// All 256 threads of the workgroup must call it (it uses __syncthreads).
template <bool TA, bool TB, int TS>
__device__ void tile_mma(const double *__restrict__ A, int64_t lda,
                         const double *__restrict__ B, int64_t ldb, int64_t m0, int64_t n0,
                         int64_t M, int64_t N, int64_t k0, int64_t k1, TileSmem<TS> &sm,
                         WaveAcc<TS> &acc) {
    constexpr int NB = TS / 32;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    const int wm = (wid >> 1) * (TS / 2), wn = (wid & 1) * (TS / 2);
    for (int64_t kc = k0; kc < k1; kc += KCH) {
#pragma unroll
        for (int r = 0; r < (KCH * TS) / BLOCK; ++r) {
            const int e = tid + BLOCK * r;
            int kk, mm;
            if (TA) { kk = e / TS; mm = e % TS; }
            else { mm = e / KCH; kk = e % KCH; }
            const int64_t gk = kc + kk, gm = m0 + mm;
            double v = 0.0;
            if (gk < k1 && gm < M) v = TA ? A[gk * lda + gm] : A[gm * lda + gk];
            sm.a[kk][mm] = v;
            int nn;
            if (TB) { nn = e / KCH; kk = e % KCH; }
            else { kk = e / TS; nn = e % TS; }
            const int64_t gk2 = kc + kk, gn = n0 + nn;
            double w = 0.0;
            if (gk2 < k1 && gn < N) w = TB ? B[gn * ldb + gk2] : B[gk2 * ldb + gn];
            sm.b[kk][nn] = w;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KCH / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double av[NB], bv[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) av[i] = sm.a[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NB; ++j) bv[j] = sm.b[kr][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc.c[i][j] = mfma_f64_16x16x4(av[i], bv[j], acc.c[i][j]);
        }
        __syncthreads();
    }
}

// Broadcast a double from `lane` (wave-uniform index) to the whole wave.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    int64_t bits = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffff), lane);
    int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// S_r(w) = sign(w) max(|w| - r, 0)  (soft-threshold operator of the paper's appendix)
__device__ __forceinline__ double soft_threshold(double w, double r) {
    const double m = fabs(w) - r;
    return m > 0.0 ? copysign(m, w) : 0.0;
}

// Sum over a wave (all 64 lanes participate).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

}  // namespace cggm
