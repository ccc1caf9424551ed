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

// One operand pair of a column-slab product: A[k][a0 + m] (m < ma) and
// B[k][b0 + n] (n < nb), k in [0, K), row-major with leading dims lda, ldb.
struct SlabPair {
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
};

// Workgroup size of the coordinate-descent tile kernels (8 waves).
constexpr int CD_BLOCK = 512;

// out[m][n] = sum over the pairs P of sum_k P.A[k][m] P.B[k][n] for a TS x TS
// output (TS = 32 or 64; entries m >= ma or n >= nb are zero), computed by
// the 8 waves of a CD_BLOCK workgroup: the output is split into 32 x 32
// quadrants and the K range into KS contiguous parts, one wave per
// (quadrant, part).  Each wave loads its MFMA operands directly from global
// memory (16 consecutive doubles per operand row, U k-steps in flight; the
// other resident waves cover the latency); the KS partial tiles are summed
// through `red` (LDS, (KS - 1) x TS x (TS + 1) doubles).  All CD_BLOCK
// threads must call it; barriers included.
template <int TS, int NPAIR, int LDO>
__device__ void slab_product(const SlabPair (&pairs)[NPAIR], int64_t K, int ma, int nb,
                             double *red, double (*out)[LDO]) {
    constexpr int NQD = TS / 32;             // quadrants per dimension
    constexpr int NQ = NQD * NQD;
    constexpr int KS = (CD_BLOCK / WAVE) / NQ;
    constexpr int U = 4;
    static_assert(KS >= 1 && NQ * KS == CD_BLOCK / WAVE, "wave split");
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int quad = wid % NQ, part = wid / NQ;
    const int mo = (quad / NQD) * 32, no = (quad % NQD) * 32;
    const int col = lane & 15, krow = lane >> 4;
    const int64_t ksteps = (K + 3) / 4;
    const int64_t s0 = (ksteps * part) / KS, s1 = (ksteps * (part + 1)) / KS;
    const bool am0 = mo + col < ma, am1 = mo + col + 16 < ma;
    const bool bn0 = no + col < nb, bn1 = no + col + 16 < nb;
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    double a0[U][2], b0[U][2];
    auto load = [&](const SlabPair &P, int64_t st, double (&a)[U][2], double (&b)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = (st + u) * 4 + krow;
            const bool kv = (st + u) < s1 && k < K;
            const double *ar = P.A + k * P.lda + mo;
            const double *br = P.B + k * P.ldb + no;
            a[u][0] = (kv && am0) ? ar[col] : 0.0;
            a[u][1] = (kv && am1) ? ar[col + 16] : 0.0;
            b[u][0] = (kv && bn0) ? br[col] : 0.0;
            b[u][1] = (kv && bn1) ? br[col + 16] : 0.0;
        }
    };
    auto mma = [&](const double (&a)[U][2], const double (&b)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = mfma_f64_16x16x4(a[u][i], b[u][j], acc[i][j]);
    };
#pragma unroll
    for (int pp = 0; pp < NPAIR; ++pp) {
        const SlabPair P = pairs[pp];
        for (int64_t st = s0; st < s1; st += U) {
            load(P, st, a0, b0);
            mma(a0, b0);
        }
    }
    constexpr int LDR = TS + 1;
    if (part == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    out[mo + i * 16 + krow + 4 * r][no + j * 16 + col] = acc[i][j][r];
    } else {
        double *rp = red + (int64_t)(part - 1) * TS * LDR;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    rp[(mo + i * 16 + krow + 4 * r) * LDR + no + j * 16 + col] = acc[i][j][r];
    }
    __syncthreads();
    if (KS > 1) {
        for (int e = tid; e < TS * TS; e += CD_BLOCK) {
            const int m = e / TS, n = e % TS;
            double v = out[m][n];
#pragma unroll
            for (int k = 0; k < KS - 1; ++k) v += red[k * TS * LDR + m * LDR + n];
            out[m][n] = v;
        }
        __syncthreads();
    }
}

template <int TS>
constexpr int slab_red_doubles() {
    return ((CD_BLOCK / WAVE) / ((TS / 32) * (TS / 32)) - 1) * TS * (TS + 1);
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
