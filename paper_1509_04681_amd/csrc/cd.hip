// cd.hip -- coordinate-descent sweeps of alternating Newton CD on gfx950.
//
// A sweep is a sequence of waves; a wave is a set of tiles (rectangles of
// coordinates) whose maintained-product rows are disjoint, so the tiles of a
// wave run concurrently without write conflicts:
//   Theta sweep (Eq. (7)): tiles are row- and column-disjoint; a tile's
//     updates touch only its rows of V = Theta Sigma.
//   Lambda direction (Eq. (6)): upper-triangle tiles whose row and column
//     index sets are pairwise disjoint; a tile's updates touch U = D Sigma
//     only in its row and column index sets.
// Inside a tile the coordinates are visited in row-major order with exact
// Gauss-Seidel semantics: the tile's gradient snapshot b is computed by an
// MFMA tile product from the maintained product, then every coordinate update
// is folded into the remaining b values of the tile through the exact
// Hessian couplings.  Tiles of the same wave see each other's updates only
// through the next wave's snapshot.
#include <math.h>

#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace cggm {

namespace {

constexpr int T = LAMBDA_TILE;    // 32
constexpr int LD = T + 1;
constexpr int TT = THETA_TILE;    // 64
constexpr int LDT = TT + 1;

// Largest number of workgroups one tile's gradient snapshot is split over.
constexpr int MAX_SPLIT = CD_MAX_SPLIT;

// Cross-workgroup sum of a tile's snapshot split over S workgroups: each
// workgroup stores its partial (out, TS x TS) in `slots` (S partials), then
// counts itself in `*cnt`; the workgroup that arrives last sums the S partials
// in slot order (so the result does not depend on arrival order) into `out`,
// resets the counter for the next wave and returns true.  The others return
// false.  All CD_BLOCK threads call it.
template <int TS, int LDO>
__device__ bool combine_partials(double (*out)[LDO], double *slots, int part, int S, int *cnt) {
    if (S == 1) return true;
    const int tid = threadIdx.x;
    double *mine = slots + (int64_t)part * TS * TS;
    for (int e = tid; e < TS * TS; e += CD_BLOCK) mine[e] = out[e / TS][e % TS];
    __threadfence();
    __syncthreads();
    __shared__ int last;
    if (tid == 0) last = (atomicAdd(cnt, 1) == S - 1);
    __syncthreads();
    if (!last) return false;
    __threadfence();
    if (tid == 0) *cnt = 0;
    for (int e = tid; e < TS * TS; e += CD_BLOCK) {
        double v = 0.0;
        for (int k = 0; k < S; ++k)
            v += __builtin_nontemporal_load(slots + (int64_t)k * TS * TS + e);
        out[e / TS][e % TS] = v;
    }
    __syncthreads();
    return true;
}

// ------------------------------------------------------------------ Theta ---
// Coordinate (i, j): along Theta_ij the Theta objective changes by
//   mu b + 1/2 a mu^2 + lamT (|Theta_ij + mu| - |Theta_ij|)
// with b = 2 Sxy_ij + 2 (Sxx V)_ij and a = 2 Sxx_ii Sigma_jj; the minimiser is
// Theta_ij <- S_{lamT/a}(Theta_ij - b/a).  Moving Theta_ij by mu changes the b
// of coordinate (i', j') by 2 Sxx_i'i Sigma_jj' mu.
__global__ __launch_bounds__(CD_BLOCK) void theta_tile_kernel(
    const TileRect *__restrict__ rects, int64_t p, int64_t q, const double *__restrict__ Sxx,
    const double *__restrict__ Sxy, const double *__restrict__ Sigma,
    const double *__restrict__ V, const double *__restrict__ GT, double *__restrict__ Theta,
    double lamT, double *__restrict__ dT, int *__restrict__ changed,
    unsigned long long *__restrict__ counters, int S, double *__restrict__ partial,
    int *__restrict__ tile_cnt) {
    const int e = blockIdx.x / S, part = blockIdx.x % S;
    const TileRect rc = rects[e];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;

    // Skip tiles without active coordinates (|G| > lambda or Theta != 0).
    int act_any = 0;
    for (int k = tid; k < TT * TT; k += CD_BLOCK) {
        const int r = k / TT, c = k % TT;
        if (r < R && c < C) {
            const int64_t idx = (int64_t)(rc.r0 + r) * q + rc.c0 + c;
            act_any |= (fabs(GT[idx]) > lamT || Theta[idx] != 0.0);
        }
    }
    if (!__syncthreads_or(act_any)) {
        if (tid == 0 && part == 0) changed[e] = 0;
        return;
    }
    __shared__ double Bs[TT][LDT];    // gradient snapshot, then corrected in place
    __shared__ union {
        double red[slab_red_doubles<TT>()];
        struct {
            double sxx[TT][LDT];      // Sxx[I, I]
            double sig[TT][LDT];      // Sigma[J, J]
        } b;
    } sh;
    auto &sxx = sh.b.sxx;
    auto &sig = sh.b.sig;

    // This workgroup's share of (Sxx V)[I, J] = Sxx[:, I]^T V[:, J] (Sxx
    // symmetric): rows [k0, k1) of the K range.
    const int64_t k0 = (p * part) / S, k1 = (p * (part + 1)) / S;
    const SlabPair pr[1] = {{Sxx + k0 * p + rc.r0, p, V + k0 * q + rc.c0, q}};
    slab_product<TT, 1, LDT>(pr, k1 - k0, R, C, sh.red, Bs);
    if (!combine_partials<TT, LDT>(Bs, partial + (int64_t)e * MAX_SPLIT * TT * TT, part, S,
                                   tile_cnt + e))
        return;                       // another workgroup finishes this tile
    if (counters && tid == 0) {
        // slabs Sxx[:, I], V[:, J]; blocks Sxx[I, I], Sigma[J, J]; Sxy, G, Theta
        // tile reads; Theta and delta writes
        atomicAdd(counters + 0, 1ull);
        atomicAdd(counters + 1, (unsigned long long)(8 * (p * (R + C) + R * R + C * C + 5 * R * C)));
        atomicAdd(counters + 2, (unsigned long long)(2 * (int64_t)R * C * p + 4 * (int64_t)R * C * C));
    }
    for (int k = tid; k < TT * TT; k += CD_BLOCK) {
        const int r = k / TT, c = k % TT;
        if (r < R && c < C) Bs[r][c] = 2.0 * Sxy[(int64_t)(rc.r0 + r) * q + rc.c0 + c] +
                                       2.0 * Bs[r][c];
        sxx[r][c] = (r < R && c < R) ? Sxx[(int64_t)(rc.r0 + r) * p + rc.r0 + c] : 0.0;
        sig[r][c] = (r < C && c < C) ? Sigma[(int64_t)(rc.c0 + r) * q + rc.c0 + c] : 0.0;
    }
    __syncthreads();
    if (wid != 0) return;

    // Exact Gauss-Seidel by one wave: lane c owns column c of the tile.
    const int c = lane;
    const bool colok = c < C;
    int any_change = 0;
    double *dTe = dT + (int64_t)e * TT * TT;
    for (int r = 0; r < R; ++r) {
        const int64_t i = rc.r0 + r;
        double th = 0.0, g = 0.0, b = 0.0, sjj = 1.0;
        if (colok) {
            th = Theta[i * q + rc.c0 + c];
            g = GT[i * q + rc.c0 + c];
            b = Bs[r][c];
            sjj = sig[c][c];
        }
        const double sii = sxx[r][r];
        const double a = 2.0 * sii * sjj;
        const bool act = colok && a > 0.0 && (fabs(g) > lamT || th != 0.0);
        uint64_t mask = __ballot(act);
        const double ainv = act ? 1.0 / a : 0.0;
        const double thr = lamT * ainv;
        double w = 0.0, mu_mine = 0.0;
        while (mask) {
            const int l = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const double cand = soft_threshold(th - b * ainv, thr) - th;
            const double mu = readlane_f64(cand, l);
            if (mu != 0.0) {
                const double s_l = colok ? sig[l][c] : 0.0;
                b += 2.0 * sii * s_l * mu;           // same-row coupling Sxx_ii Sigma_lc
                w += s_l * mu;
                if (c == l) {
                    mu_mine = mu;
                    th += mu;
                }
                any_change = 1;
            }
        }
        if (colok) {
            Theta[i * q + rc.c0 + c] = th;
            dTe[r * TT + c] = mu_mine;
            // later rows: b[r2][c] += 2 Sxx[r2][r] sum_l mu_l Sigma[l][c]
            for (int r2 = r + 1; r2 < R; ++r2) Bs[r2][c] += 2.0 * sxx[r2][r] * w;
        }
    }
    if (lane == 0) changed[e] = any_change;
}

// Out[m][n] += sum_k op(Delta)[m][k] S[k][n] for m < R, k < Kd and the
// columns [c_begin, c_end) of a row block (the maintained-product update of a
// tile).  op(Delta)[m][k] = Delta[m * TK + k], or Delta[k * TK + m] when
// `trans`.  Delta is staged in LDS once; each of the 4 waves owns 16 columns of
// every 64-column chunk, loads its S operands straight from global memory (one
// 128-byte row segment per k-step) and read-modify-writes Out from the MFMA
// accumulators.  All BLOCK threads call it.
template <int TR, int TK>
__device__ void rowblock_update(const double *__restrict__ Delta, bool trans, int R, int Kd,
                                const double *__restrict__ S, int64_t lds,
                                double *__restrict__ Out, int64_t ldo, int64_t c_begin,
                                int64_t c_end, double (*dl)[TR + 2]) {
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    for (int e = tid; e < TK * TR; e += BLOCK) {
        const int k = e / TR, m = e % TR;
        dl[k][m] = (m < R && k < Kd) ? (trans ? Delta[k * TK + m] : Delta[m * TK + k]) : 0.0;
    }
    __syncthreads();
    constexpr int KST = TK / 4, NI = TR / 16;
    const int col = lane & 15, krow = lane >> 4;
    // Operands of one 64-column chunk: S values for the MFMA B operand and the
    // current Out values this lane updates.  The next chunk's loads are issued
    // before the current chunk's MFMAs so their latency overlaps.
    struct Chunk {
        double bv[KST];
        double ov[NI][4];
    };
    auto load = [&](int64_t c0, Chunk &ch) {
        const int64_t n = c0 + wid * 16 + col;
        const bool nv = c0 < c_end && n < c_end;
#pragma unroll
        for (int ks = 0; ks < KST; ++ks) {
            const int k = ks * 4 + krow;
            ch.bv[ks] = (nv && k < Kd) ? S[(int64_t)k * lds + n] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = i * 16 + krow + 4 * r;
                ch.ov[i][r] = (nv && m < R) ? Out[(int64_t)m * ldo + n] : 0.0;
            }
    };
    auto apply = [&](int64_t c0, const Chunk &ch) {
        const int64_t n = c0 + wid * 16 + col;
        const bool nv = n < c_end;
        v4d acc[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i)
            acc[i] = v4d{ch.ov[i][0], ch.ov[i][1], ch.ov[i][2], ch.ov[i][3]};
#pragma unroll
        for (int ks = 0; ks < KST; ++ks)
#pragma unroll
            for (int i = 0; i < NI; ++i)
                acc[i] = mfma_f64_16x16x4(dl[ks * 4 + krow][i * 16 + col], ch.bv[ks], acc[i]);
        if (nv) {
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = i * 16 + krow + 4 * r;
                    if (m < R) Out[(int64_t)m * ldo + n] = acc[i][r];
                }
        }
    };
    Chunk a, b;
    load(c_begin, a);
    for (int64_t c0 = c_begin; c0 < c_end; c0 += 128) {
        load(c0 + 64, b);
        apply(c0, a);
        load(c0 + 128, a);
        if (c0 + 64 < c_end) apply(c0 + 64, b);
    }
}

constexpr int UPD_CHUNKS = 4;   // 64-column chunks per update workgroup

// V[I, :] += dTheta[I, J] Sigma[J, :] for every changed tile of the wave.
__global__ __launch_bounds__(BLOCK) void theta_v_update_kernel(
    const TileRect *__restrict__ rects, int64_t q, const double *__restrict__ Sigma,
    const double *__restrict__ dT, const int *__restrict__ changed, double *__restrict__ V) {
    const int e = blockIdx.y;
    if (!changed[e]) return;
    const TileRect rc = rects[e];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int64_t c_begin = (int64_t)blockIdx.x * 64 * UPD_CHUNKS;
    const int64_t c_end = std::min<int64_t>(q, c_begin + 64 * UPD_CHUNKS);
    __shared__ double dl[TT][TT + 2];
    rowblock_update<TT, TT>(dT + (int64_t)e * TT * TT, false, R, C, Sigma + (int64_t)rc.c0 * q,
                            q, V + (int64_t)rc.r0 * q, q, c_begin, c_end, dl);
}

// ----------------------------------------------------------------- Lambda ---
// Quadratic model of Eq. (6): gbar(D) = tr(G D) + 1/2 tr(D S D S) + tr(D S D P)
// (S = Sigma, P = Psi; Hessian S (x) (S + 2 P), Eq. (4)).  Moving the pair
// D_ij = D_ji by mu (i != j) changes gbar + penalty by
//   2 [mu b + 1/2 a mu^2 + lamL (|c + mu| - |c|)],
//   a = S_ij^2 + S_ii S_jj + S_ii P_jj + S_jj P_ii + 2 S_ij P_ij,
//   b = G_ij + (S D S)_ij + (P D S)_ij + (P D S)_ji = G_ij + (SP U)_ij + (P U)_ji,
// with U = D S, SP = S + P and c = Lambda_ij + D_ij; a diagonal coordinate
// has a = S_ii^2 + 2 S_ii P_ii and the same b.  The minimiser is
// mu = -c + S_{lamL/a}(c - b/a).  The move changes U in rows i and j
// (U_i. += mu S_j., U_j. += mu S_i.; only row i when i == j), hence the b of
// coordinate (i', j') by
//   mu_e [SP_i'i S_lj' + SP_i'l S_ij' + P_ij' S_i'l + P_lj' S_ii']
// for a move at (i, l), with mu_e = mu (l != i) or mu / 2 (l == i).
__global__ __launch_bounds__(CD_BLOCK) void lambda_tile_kernel(
    const TileRect *__restrict__ rects, int64_t q, const double *__restrict__ Sigma,
    const double *__restrict__ Psi, const double *__restrict__ SP,
    const double *__restrict__ GL, const double *__restrict__ Lam, double lamL,
    double *__restrict__ D, const double *__restrict__ U, double *__restrict__ dD,
    int *__restrict__ changed, unsigned long long *__restrict__ counters, int S,
    double *__restrict__ partial, int *__restrict__ tile_cnt) {
    const int e = blockIdx.x / S, part = blockIdx.x % S;
    const TileRect rc = rects[e];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const bool diag = rc.r0 == rc.c0;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;

    int act_any = 0;
    for (int k = tid; k < T * T; k += CD_BLOCK) {
        const int r = k / T, c = k % T;
        if (r < R && c < C && (!diag || c >= r)) {
            const int64_t idx = (int64_t)(rc.r0 + r) * q + rc.c0 + c;
            act_any |= (fabs(GL[idx]) > lamL || Lam[idx] != 0.0);
        }
    }
    if (!__syncthreads_or(act_any)) {
        if (tid == 0 && part == 0) changed[e] = 0;
        return;
    }
    __shared__ double Bs[T][LD];
    __shared__ union {
        double red[slab_red_doubles<T>()];
        struct {
            double sII[T][LD], pII[T][LD], sJJ[T][LD], pJJ[T][LD], sIJ[T][LD], pIJ[T][LD];
        } b;
    } sh;
    auto &sII = sh.b.sII;
    auto &pII = sh.b.pII;
    auto &sJJ = sh.b.sJJ;
    auto &pJJ = sh.b.pJJ;
    auto &sIJ = sh.b.sIJ;
    auto &pIJ = sh.b.pIJ;

    // b snapshot: G + (SP U)[I, J] + ((Psi U)[J, I])^T
    //   = G + SP[:, I]^T U[:, J] + U[:, I]^T Psi[:, J]   (SP, Psi symmetric);
    // this workgroup sums the rows [k0, k1) of the K range.
    const int64_t k0 = (q * part) / S, k1 = (q * (part + 1)) / S;
    const SlabPair pr[2] = {{SP + k0 * q + rc.r0, q, U + k0 * q + rc.c0, q},
                            {U + k0 * q + rc.r0, q, Psi + k0 * q + rc.c0, q}};
    slab_product<T, 2, LD>(pr, k1 - k0, R, C, sh.red, Bs);
    if (!combine_partials<T, LD>(Bs, partial + (int64_t)e * MAX_SPLIT * T * T, part, S,
                                 tile_cnt + e))
        return;                       // another workgroup finishes this tile
    if (counters && tid == 0) {
        // slabs SP[:, I], U[:, J], U[:, I], Psi[:, J]; six Sigma / Psi blocks;
        // G and Lambda tile reads; D (both triangles) and delta writes
        atomicAdd(counters + 0, 1ull);
        atomicAdd(counters + 1, (unsigned long long)(8 * (2 * q * (R + C) + 2 * R * R + 2 * C * C +
                                                         7 * R * C)));
        atomicAdd(counters + 2, (unsigned long long)(4 * (int64_t)R * C * q + 16 * (int64_t)R * C * C));
    }
    for (int k = tid; k < T * T; k += CD_BLOCK) {
        const int r = k / T, c = k % T;
        const bool ii = r < R && c < R, jj = r < C && c < C, ij = r < R && c < C;
        if (ij) Bs[r][c] += GL[(int64_t)(rc.r0 + r) * q + rc.c0 + c];
        sII[r][c] = ii ? Sigma[(int64_t)(rc.r0 + r) * q + rc.r0 + c] : 0.0;
        pII[r][c] = ii ? Psi[(int64_t)(rc.r0 + r) * q + rc.r0 + c] : 0.0;
        sJJ[r][c] = jj ? Sigma[(int64_t)(rc.c0 + r) * q + rc.c0 + c] : 0.0;
        pJJ[r][c] = jj ? Psi[(int64_t)(rc.c0 + r) * q + rc.c0 + c] : 0.0;
        sIJ[r][c] = ij ? Sigma[(int64_t)(rc.r0 + r) * q + rc.c0 + c] : 0.0;
        pIJ[r][c] = ij ? Psi[(int64_t)(rc.r0 + r) * q + rc.c0 + c] : 0.0;
    }
    __syncthreads();
    if (wid != 0) return;

    const int c = lane;
    const bool inC = c < C;
    int any_change = 0;
    double *dDe = dD + (int64_t)e * T * T;
    for (int r = 0; r < R; ++r) {
        const int64_t i = rc.r0 + r;
        const bool colok = inC && (!diag || c >= r);
        double lamv = 0.0, g = 0.0, b = 0.0, s_ij = 0.0, p_ij = 0.0, s_jj = 0.0, p_jj = 0.0;
        if (inC) {
            lamv = Lam[i * q + rc.c0 + c];
            g = GL[i * q + rc.c0 + c];
            b = Bs[r][c];
            s_ij = sIJ[r][c];
            p_ij = pIJ[r][c];
            s_jj = sJJ[c][c];
            p_jj = pJJ[c][c];
        }
        const double sii = sII[r][r], pii = pII[r][r], spii = sii + pii;
        const bool self = diag && c == r;
        const double a = self ? sii * sii + 2.0 * sii * pii
                              : s_ij * s_ij + sii * s_jj + sii * p_jj + s_jj * pii +
                                    2.0 * s_ij * p_ij;
        const bool act = colok && a > 0.0 && (fabs(g) > lamL || lamv != 0.0);
        uint64_t mask = __ballot(act);
        const double ainv = act ? 1.0 / a : 0.0;
        const double thr = lamL * ainv;
        double w1 = 0.0, w4 = 0.0, mu_mine = 0.0;
        while (mask) {
            const int l = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            // c = Lambda_ij + D_ij with D_ij = 0 until the coordinate is visited
            const double cand = soft_threshold(lamv - b * ainv, thr) - lamv;
            const double mu = readlane_f64(cand, l);
            if (mu != 0.0) {
                const double mue = (diag && l == r) ? 0.5 * mu : mu;
                const double s_il = readlane_f64(s_ij, l), p_il = readlane_f64(p_ij, l);
                const double sJl = sJJ[l][c], pJl = pJJ[l][c];
                b += mue * (spii * sJl + (s_il + p_il) * s_ij + p_ij * s_il + pJl * sii);
                w1 += mue * sJl;
                w4 += mue * pJl;
                if (c == l) mu_mine = mu;
                any_change = 1;
            }
        }
        if (colok) {
            D[i * q + rc.c0 + c] = mu_mine;
            D[(int64_t)(rc.c0 + c) * q + i] = mu_mine;
        }
        if (inC) {
            if (!diag) {
                dDe[r * T + c] = mu_mine;
            } else if (c >= r) {                 // symmetric delta of a diagonal tile
                dDe[r * T + c] = mu_mine;
                dDe[c * T + r] = mu_mine;
            }
        }
        // Corrections of the later rows r2 of the tile:
        //   b[r2][c] += SP[r2][r] w1_c + S[r][c] w2_r2 + P[r][c] w3_r2 + S[r][r2] w4_c
        //   w2_r2 = sum_l SP[r2][l] mu_e,l,   w3_r2 = sum_l S[r2][l] mu_e,l.
        const double mue_mine = (diag && c == r) ? 0.5 * mu_mine : mu_mine;
        uint64_t moved = __ballot(mu_mine != 0.0);
        if (moved == 0) continue;
        double w2 = 0.0, w3 = 0.0;            // lane r2 accumulates row r2's values
        const int r2l = lane;
        while (moved) {
            const int l = __ffsll((unsigned long long)moved) - 1;
            moved &= moved - 1;
            const double m = readlane_f64(mue_mine, l);
            if (r2l < R) {
                const double sv = sIJ[r2l][l];
                w2 += (sv + pIJ[r2l][l]) * m;
                w3 += sv * m;
            }
        }
        for (int r2 = r + 1; r2 < R; ++r2) {
            const double w2r = readlane_f64(w2, r2), w3r = readlane_f64(w3, r2);
            if (inC)
                Bs[r2][c] += (sII[r2][r] + pII[r2][r]) * w1 + s_ij * w2r + p_ij * w3r +
                             sII[r][r2] * w4;
        }
    }
    if (lane == 0) changed[e] = any_change;
}

// U[I, :] += dD Sigma[J, :] and U[J, :] += dD^T Sigma[I, :] (off-diagonal
// tiles), or U[I, :] += dD_sym Sigma[I, :] (diagonal tiles).
__global__ __launch_bounds__(BLOCK) void lambda_u_update_kernel(
    const TileRect *__restrict__ rects, int64_t q, const double *__restrict__ Sigma,
    const double *__restrict__ dD, const int *__restrict__ changed, double *__restrict__ U) {
    const int e = blockIdx.y, half = blockIdx.z;
    if (!changed[e]) return;
    const TileRect rc = rects[e];
    const bool diag = rc.r0 == rc.c0;
    if (diag && half == 1) return;
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int64_t c_begin = (int64_t)blockIdx.x * 64 * UPD_CHUNKS;
    const int64_t c_end = std::min<int64_t>(q, c_begin + 64 * UPD_CHUNKS);
    __shared__ double dl[T][T + 2];
    const double *dDe = dD + (int64_t)e * T * T;
    if (half == 0)
        rowblock_update<T, T>(dDe, false, R, C, Sigma + (int64_t)rc.c0 * q, q,
                              U + (int64_t)rc.r0 * q, q, c_begin, c_end, dl);
    else
        rowblock_update<T, T>(dDe, true, C, R, Sigma + (int64_t)rc.r0 * q, q,
                              U + (int64_t)rc.c0 * q, q, c_begin, c_end, dl);
}

// Workgroups per tile snapshot: about 1024 workgroups per wave, at most
// MAX_SPLIT, and at least 256 rows of K per workgroup.
int snapshot_split(int nrect, int64_t K) {
    int S = (1024 + nrect - 1) / nrect;
    S = std::min(S, MAX_SPLIT);
    S = (int)std::min<int64_t>(S, std::max<int64_t>(1, K / 256));
    return std::max(S, 1);
}

}  // namespace

void theta_wave(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t p, int64_t q,
                const double *Sxx, const double *Sxy, const double *Sigma, double *V,
                const double *GT, double *Theta, double lamT, double *dT, int *changed,
                const CdScratch &scr, const WaveProbe *probe) {
    if (nrect <= 0) return;
    const int S = snapshot_split(nrect, p);
    if (probe) CGGM_HIP(hipEventRecord(probe->start, s));
    theta_tile_kernel<<<nrect * S, CD_BLOCK, 0, s>>>(rects_dev, p, q, Sxx, Sxy, Sigma, V, GT,
                                                     Theta, lamT, dT, changed,
                                                     probe ? probe->counters : nullptr, S,
                                                     scr.partial, scr.tile_cnt);
    CGGM_LAUNCH_CHECK();
    if (probe) CGGM_HIP(hipEventRecord(probe->stop, s));
    const int64_t cols_per_wg = 64 * UPD_CHUNKS;
    dim3 grid((unsigned)((q + cols_per_wg - 1) / cols_per_wg), (unsigned)nrect);
    theta_v_update_kernel<<<grid, BLOCK, 0, s>>>(rects_dev, q, Sigma, dT, changed, V);
    CGGM_LAUNCH_CHECK();
}

void lambda_wave(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t q,
                 const double *Sigma, const double *Psi, const double *SP, const double *GL,
                 const double *Lam, double lamL, double *D, double *U, double *dD,
                 int *changed, const CdScratch &scr, const WaveProbe *probe) {
    if (nrect <= 0) return;
    const int S = snapshot_split(nrect, q);
    if (probe) CGGM_HIP(hipEventRecord(probe->start, s));
    lambda_tile_kernel<<<nrect * S, CD_BLOCK, 0, s>>>(rects_dev, q, Sigma, Psi, SP, GL, Lam,
                                                      lamL, D, U, dD, changed,
                                                      probe ? probe->counters : nullptr, S,
                                                      scr.partial, scr.tile_cnt);
    CGGM_LAUNCH_CHECK();
    if (probe) CGGM_HIP(hipEventRecord(probe->stop, s));
    const int64_t cols_per_wg = 64 * UPD_CHUNKS;
    dim3 grid((unsigned)((q + cols_per_wg - 1) / cols_per_wg), (unsigned)nrect, 2);
    lambda_u_update_kernel<<<grid, BLOCK, 0, s>>>(rects_dev, q, Sigma, dD, changed, U);
    CGGM_LAUNCH_CHECK();
}

}  // namespace cggm
