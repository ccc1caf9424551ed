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
// Gauss-Seidel semantics: the tile's gradient snapshot b is computed from the
// maintained product, then every coordinate update is folded into the
// remaining b values of the tile through the exact Hessian couplings.  Tiles
// of the same wave see each other's updates only through the next wave's
// snapshot.
//
// A wave runs four kernels:
//   1. snapshot: the MFMA column-slab products of every tile, split over the
//      K range into parts, one wavefront per (tile, 64x32 block, K part);
//      partial tiles go to a scratch buffer;
//   2. the sum of each tile's partials in part order (deterministic);
//   3. Gauss-Seidel: one workgroup per tile adds the gradient term to the
//      summed snapshot and runs the exact in-tile CD;
//   4. update of the maintained product's rows with the tile deltas.
// Which tiles have active coordinates is decided once per sweep (the screen
// uses the gradient and the parameters at the start of the sweep).
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace cggm {

namespace {

constexpr int T = LAMBDA_TILE;    // 64
constexpr int TT = THETA_TILE;    // 64
// Rows with at least this many active coordinates take the unrolled
// register-operand scan in the Theta Gauss-Seidel kernel; sparser rows iterate
// over their active lanes only.
constexpr int GS_DENSE_ROW = 16;
constexpr int LDT = TT + 1;

// ----------------------------------------------------------------- activity --
// active[r] = the number of coordinates of rect r with |G| > lam or P != 0
// (upper triangle only for the diagonal rects of Lambda); nonzero = active.
__global__ __launch_bounds__(BLOCK) void tile_activity_kernel(const TileRect *__restrict__ rects,
                                                              int64_t ld, const double *__restrict__ G,
                                                              const double *__restrict__ P,
                                                              double lam, int upper,
                                                              int *__restrict__ active) {
    const TileRect rc = rects[blockIdx.x];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const bool diag = upper && rc.r0 == rc.c0;
    __shared__ int count;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    int mine = 0;
    for (int k = threadIdx.x; k < R * C; k += BLOCK) {
        const int r = k / C, c = k % C;
        if (!diag || c >= r) {
            const int64_t idx = (int64_t)(rc.r0 + r) * ld + rc.c0 + c;
            mine += (fabs(G[idx]) > lam || P[idx] != 0.0) ? 1 : 0;
        }
    }
    if (mine) atomicAdd(&count, mine);
    __syncthreads();
    if (threadIdx.x == 0) active[blockIdx.x] = count;
}

// ----------------------------------------------------------------- snapshot --
// Operand pairs of the snapshot products: out[m][n] += sum_k A[k][r0 + m] B[k][c0 + n]
// (A, B symmetric or stored so that the tile's rows/columns are column slabs).
// E = double: FP64 matrix cores and accumulation (snapshot64_block); E = float:
// the FP32 copies of the mixed mode (snapshot32_block).
template <int NPAIR, class E>
struct SnapArgs {
    const E *A[NPAIR];
    int64_t lda[NPAIR];
    const E *B[NPAIR];
    int64_t ldb[NPAIR];
};

// One wavefront per workgroup computes one WM x WN block of one tile's
// snapshot over one part of the K range, loading its MFMA operands straight
// from HBM (16 consecutive doubles per operand row, U k-steps in flight) and
// writing the partial from its accumulators.  No LDS, so many wavefronts stay
// resident per CU to cover the memory latency.
//
// Workgroups are dealt to the 8 XCDs round robin by block index, and each XCD
// has its own L2.  The blocks of one (tile, part) read the same operand
// column slabs, so their block indices are chosen congruent mod 8: later
// readers of a slab hit the L2 of the first.
constexpr int NXCD = 8;
inline int64_t snapshot_blocks(int64_t groups, int blocks_per_group) {
    return (groups + NXCD - 1) / NXCD * NXCD * blocks_per_group;
}

// A buffer resource over `bytes` bytes from p (raw addressing, 32-bit data
// format): a load at an offset at or past `bytes` returns zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}

// Block of one wavefront: 64 x 32 (6 operand loads per 8 MFMAs per k-step),
// two register batches of U = 4 k-steps (one in flight while the other is
// multiplied); about 170 VGPRs + 64 AGPRs, two waves per SIMD.
constexpr int SNAP_WM = 64, SNAP_WN = 32, SNAP_U = 4;
template <int TS>
constexpr int snap_blocks_per_tile() {
    return (TS / SNAP_WM) * (TS / SNAP_WN);
}
// Block `blk` of part `s` of tile e from FP64 operands, every load predicated
// on the K range and the tile's extent.  (Reading the part's rows through
// buffer resources instead, as the FP32 block does, measured 3% slower here:
// 1308 against 1268 us per wave at q = 20000, 188 against 236 VGPRs, two
// waves per SIMD either way.)
template <int TS, int NPAIR>
__device__ __forceinline__ void snapshot64_block(const TileRect rc, int e, int s, int blk, int S,
                                                 int64_t K, const SnapArgs<NPAIR, double> &args,
                                                 double *__restrict__ partial) {
    constexpr int WM = SNAP_WM, WN = SNAP_WN, U = SNAP_U;
    constexpr int NBN = TS / WN, MI = WM / 16, NJ = WN / 16;
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int mo = (blk / NBN) * WM, no = (blk % NBN) * WN;
    if (mo >= R || no >= C) return;                  // block outside a ragged tile
    const int lane = threadIdx.x, col = lane & 15, krow = lane >> 4;
    const int64_t ksteps = (K + 3) / 4;
    const int64_t s0 = (ksteps * s) / S, s1 = (ksteps * (s + 1)) / S;
    bool am[MI], bn[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i) am[i] = mo + i * 16 + col < R;
#pragma unroll
    for (int j = 0; j < NJ; ++j) bn[j] = no + j * 16 + col < C;
    v4d acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int pp = 0; pp < NPAIR; ++pp) {
        const int64_t lda = args.lda[pp], ldb = args.ldb[pp];
        // Two register batches: the loads of the next batch are in flight
        // while the current one is multiplied (loads past the K range read
        // zeros and multiply zeros).
        double a[2][U][MI], b[2][U][NJ];
#define SNAP_MMA(BUF_)                                                                   \
    _Pragma("unroll") for (int u = 0; u < U; ++u)                                        \
        _Pragma("unroll") for (int i = 0; i < MI; ++i)                                   \
            _Pragma("unroll") for (int j = 0; j < NJ; ++j)                               \
                acc[i][j] = mfma_f64_16x16x4(a[BUF_][u][i], b[BUF_][u][j], acc[i][j]);
        const double *A = args.A[pp] + rc.r0 + mo;
        const double *B = args.B[pp] + rc.c0 + no;
#define SNAP_LOAD(BUF_, ST0)                                                             \
    _Pragma("unroll") for (int u = 0; u < U; ++u) {                                      \
        const int64_t k = ((ST0) + u) * 4 + krow;                                        \
        const bool kv = ((ST0) + u) < s1 && k < K;                                       \
        _Pragma("unroll") for (int i = 0; i < MI; ++i) a[BUF_][u][i] =                   \
            (kv && am[i]) ? A[k * lda + col + i * 16] : 0.0;                             \
        _Pragma("unroll") for (int j = 0; j < NJ; ++j) b[BUF_][u][j] =                   \
            (kv && bn[j]) ? B[k * ldb + col + j * 16] : 0.0;                             \
    }
        SNAP_LOAD(0, s0)
        for (int64_t st = s0; st < s1; st += 2 * U) {
            SNAP_LOAD(1, st + U)
            SNAP_MMA(0)
            SNAP_LOAD(0, st + 2 * U)
            SNAP_MMA(1)
        }
#undef SNAP_LOAD
#undef SNAP_MMA
    }
    double *out = partial + ((int64_t)e * S + s) * TS * TS;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(mo + i * 16 + krow + 4 * r) * TS + no + j * 16 + col] = acc[i][j][r];
}

// ------------------------------------------------ FP32 operands (mixed mode) --
// The mixed-mode snapshot and update read FP32 copies of the streamed
// operands (row length a multiple of 4, padding zero) and multiply on the
// FP32 matrix cores: v_mfma_f32_16x16x4f32, where lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16].
// So that a lane loads 16 (8) bytes at once, MFMA block i of a 64-row block
// takes the rows {4 c + i} and block j of a 32-column block the columns
// {2 c + j} (c = 0..15): one float4 (float2) load gives a lane its values for
// all four (two) blocks.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma_f32_16x16x4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Up to four (two) consecutive floats from p; entries at or past `valid` are
// zero and not read.  A full vector is read only when all of it is valid.
__device__ __forceinline__ f32x4 load4_upto(const float *p, int valid) {
    if (valid >= 4) return *reinterpret_cast<const f32x4 *>(p);
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (valid > 0) v[0] = p[0];
    if (valid > 1) v[1] = p[1];
    if (valid > 2) v[2] = p[2];
    return v;
}
__device__ __forceinline__ f32x2 load2_upto(const float *p, int valid) {
    if (valid >= 2) return *reinterpret_cast<const f32x2 *>(p);
    f32x2 v = {0.f, 0.f};
    if (valid > 0) v[0] = p[0];
    return v;
}

// The snapshot of snapshot64_block from FP32 operands (same blocks, parts and
// XCD mapping), FP32 accumulation, FP64 partials: block `blk` of part `s` of
// tile e.  BUF (every load offset of the part below 2^31 bytes, and every
// ragged tile ending at the matrix edge, whose FP32 copy is zero-padded to
// its row length): the operands are read through buffer resources that end
// at the part's last row, so the loads past the part and outside the tile
// return zeros with no predicate and no branch.  Otherwise the loads are
// predicated on the K range and on the tile's valid rows and columns.
template <int TS, int NPAIR, bool BUF>
__device__ __forceinline__ void snapshot32_block(const TileRect rc, int e, int s, int blk, int S,
                                                 int64_t K, const SnapArgs<NPAIR, float> &args,
                                                 double *__restrict__ partial) {
    constexpr int WM = SNAP_WM, WN = SNAP_WN, U = SNAP_U;
    static_assert(WM == 64 && WN == 32, "float4 rows and float2 columns per lane");
    constexpr int NBN = TS / WN;
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int mo = (blk / NBN) * WM, no = (blk % NBN) * WN;
    if (mo >= R || no >= C) return;                  // block outside a ragged tile
    const int lane = threadIdx.x, col = lane & 15, krow = lane >> 4;
    const int ra = R - mo - 4 * col;                 // valid rows of this lane's float4
    const int cb = C - no - 2 * col;                 // valid columns of its float2
    const int64_t ksteps = (K + 3) / 4;
    const int64_t s0 = (ksteps * s) / S, s1 = (ksteps * (s + 1)) / S;
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int pp = 0; pp < NPAIR; ++pp) {
        const int64_t lda = args.lda[pp], ldb = args.ldb[pp];
        f32x4 a[2][U];
        f32x2 b[2][U];
#define SNAP32_MMA(BUF_)                                                                 \
    _Pragma("unroll") for (int u = 0; u < U; ++u)                                        \
        _Pragma("unroll") for (int i = 0; i < 4; ++i)                                    \
            _Pragma("unroll") for (int j = 0; j < 2; ++j)                                \
                acc[i][j] = mfma_f32_16x16x4(a[BUF_][u][i], b[BUF_][u][j], acc[i][j]);
        if (BUF) {
            // rows [k0, k1) of the operands; each offset is in the per-lane
            // operand, which the range check covers
            const int64_t k0 = 4 * s0, k1 = std::min<int64_t>(K, 4 * s1);
            const __amdgpu_buffer_rsrc_t rA =
                buffer_rsrc(args.A[pp] + k0 * lda + rc.r0 + mo, (int)((k1 - k0) * lda * 4));
            const __amdgpu_buffer_rsrc_t rB =
                buffer_rsrc(args.B[pp] + k0 * ldb + rc.c0 + no, (int)((k1 - k0) * ldb * 4));
            // a lane whose vector lies wholly outside a ragged tile starts at
            // the buffer's end (its loads read zeros); one that straddles the
            // tile's last column reads the zero padding past the matrix edge
            const unsigned va = ra > 0 ? (unsigned)(krow * lda * 4 + 16 * col)
                                       : (unsigned)((k1 - k0) * lda * 4);
            const unsigned vb = cb > 0 ? (unsigned)(krow * ldb * 4 + 8 * col)
                                       : (unsigned)((k1 - k0) * ldb * 4);
            const unsigned sa = (unsigned)(16 * lda), sb = (unsigned)(16 * ldb);  // per k-step
#define SNAP32_BLOAD(BUF_, ST0)                                                          \
    _Pragma("unroll") for (int u = 0; u < U; ++u) {                                      \
        const unsigned r = (unsigned)((ST0) - s0) + u;                                   \
        a[BUF_][u] = __builtin_bit_cast(                                                 \
            f32x4, __builtin_amdgcn_raw_buffer_load_b128(rA, (int)(va + r * sa), 0, 0)); \
        b[BUF_][u] = __builtin_bit_cast(                                                 \
            f32x2, __builtin_amdgcn_raw_buffer_load_b64(rB, (int)(vb + r * sb), 0, 0));  \
    }
            SNAP32_BLOAD(0, s0)
            for (int64_t st = s0; st < s1; st += 2 * U) {
                SNAP32_BLOAD(1, st + U)
                SNAP32_MMA(0)
                SNAP32_BLOAD(0, st + 2 * U)
                SNAP32_MMA(1)
            }
#undef SNAP32_BLOAD
        } else {
            const float *A = args.A[pp] + rc.r0 + mo + 4 * col;
            const float *B = args.B[pp] + rc.c0 + no + 2 * col;
#define SNAP32_LOAD(BUF_, ST0)                                                           \
    _Pragma("unroll") for (int u = 0; u < U; ++u) {                                      \
        const int64_t k = ((ST0) + u) * 4 + krow;                                        \
        const bool kv = ((ST0) + u) < s1 && k < K;                                       \
        a[BUF_][u] = kv ? load4_upto(A + k * lda, ra) : f32x4{0.f, 0.f, 0.f, 0.f};       \
        b[BUF_][u] = kv ? load2_upto(B + k * ldb, cb) : f32x2{0.f, 0.f};                 \
    }
            SNAP32_LOAD(0, s0)
            for (int64_t st = s0; st < s1; st += 2 * U) {
                SNAP32_LOAD(1, st + U)
                SNAP32_MMA(0)
                SNAP32_LOAD(0, st + 2 * U)
                SNAP32_MMA(1)
            }
#undef SNAP32_LOAD
        }
#undef SNAP32_MMA
    }
    double *out = partial + ((int64_t)e * S + s) * TS * TS;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(mo + 4 * (4 * krow + r) + i) * TS + no + 2 * col + j] = (double)acc[i][j][r];
}

template <int TS, int NPAIR, class E, bool BUF>
__device__ __forceinline__ void snapshot_block(const TileRect rc, int e, int s, int blk, int S,
                                               int64_t K, const SnapArgs<NPAIR, E> &args,
                                               double *__restrict__ partial) {
    if constexpr (std::is_same<E, float>::value)
        snapshot32_block<TS, NPAIR, BUF>(rc, e, s, blk, S, K, args, partial);
    else
        snapshot64_block<TS, NPAIR>(rc, e, s, blk, S, K, args, partial);
}

// Every active tile, one wavefront per block.
template <int TS, int NPAIR, class E, bool BUF>
__global__ __launch_bounds__(WAVE) void snapshot_kernel(const TileRect *__restrict__ rects,
                                                        const int *__restrict__ active, int S,
                                                        int nrect, int64_t K,
                                                        SnapArgs<NPAIR, E> args,
                                                        double *__restrict__ partial) {
    constexpr int NB = snap_blocks_per_tile<TS>();
    const int64_t wg = blockIdx.x;
    const int64_t rest = wg / NXCD;
    const int blk = (int)(rest % NB);
    const int64_t t = (rest / NB) * NXCD + wg % NXCD;   // (tile, part) group
    if (t >= (int64_t)nrect * S) return;
    const int s = (int)(t % S);
    const int e = (int)(t / S);
    if (!active[e]) return;
    snapshot_block<TS, NPAIR, E, BUF>(rects[e], e, s, blk, S, K, args, partial);
}

// Launch of the snapshot of one wave with `full` tiles of TS x TS (-1: not
// known): for FP32 operands the buffer path when there is one (the schedule
// has TS-edge tiles, so every other tile ends at the matrix edge) and every
// load offset of a part stays below 2^31 bytes, else the predicated path.
template <int TS, int NPAIR, class E>
void snapshot(hipStream_t st, const TileRect *rects, const int *active, int S, int nrect,
              int64_t K, const SnapArgs<NPAIR, E> &args, int full, double *partial) {
    constexpr int NB = snap_blocks_per_tile<TS>();
    int64_t ld = 0;
    for (int pp = 0; pp < NPAIR; ++pp) ld = std::max(ld, std::max(args.lda[pp], args.ldb[pp]));
    // rows a part's loads may reach: its k-steps plus the 3 U k-steps the
    // register batches run past its end
    const int64_t rows = ((K + 3) / 4 / S + 1 + 3 * SNAP_U) * 4;
    const unsigned nsb = (unsigned)snapshot_blocks((int64_t)nrect * S, NB);
    if constexpr (std::is_same<E, float>::value) {
        if (full > 0 && (rows + 1) * ld * (int64_t)sizeof(E) < ((int64_t)1 << 31)) {
            snapshot_kernel<TS, NPAIR, E, true><<<nsb, WAVE, 0, st>>>(rects, active, S, nrect, K,
                                                                       args, partial);
            CGGM_LAUNCH_CHECK();
            return;
        }
    }
    snapshot_kernel<TS, NPAIR, E, false><<<nsb, WAVE, 0, st>>>(rects, active, S, nrect, K, args,
                                                                partial);
    CGGM_LAUNCH_CHECK();
}

// Sum of the S partial snapshots of every active tile, in part order
// (deterministic), into part 0; one thread per tile entry, eight loads in
// flight.  Entries outside a ragged tile are summed too and never read.
template <int TS>
__global__ __launch_bounds__(BLOCK) void snapshot_sum_kernel(const int *__restrict__ active,
                                                             int S, double *__restrict__ partial) {
    const int e = blockIdx.y;
    if (!active[e]) return;
    const int k = blockIdx.x * BLOCK + threadIdx.x;
    double *base = partial + (int64_t)e * S * TS * TS + k;
    double v = base[0];
    int s = 1;
    for (; s + 8 <= S; s += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = base[(int64_t)(s + u) * TS * TS];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t[u];
    }
    for (; s < S; ++s) v += base[(int64_t)s * TS * TS];
    base[0] = v;
}

template <int TS>
void sum_snapshots(hipStream_t st, const int *active, int nrect, int S, double *partial) {
    static_assert((TS * TS) % BLOCK == 0, "whole blocks per tile");
    if (S <= 1) return;
    snapshot_sum_kernel<TS><<<dim3(TS * TS / BLOCK, nrect), BLOCK, 0, st>>>(active, S, partial);
    CGGM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ Theta ---
// Coordinate (i, j): along Theta_ij the Theta objective changes by
//   mu b + 1/2 a mu^2 + lamT (|Theta_ij + mu| - |Theta_ij|)
// with b = 2 Sxy_ij + 2 (Sxx V)_ij and a = 2 Sxx_ii Sigma_jj; the minimiser is
// Theta_ij <- S_{lamT/a}(Theta_ij - b/a).  Moving Theta_ij by mu changes the b
// of coordinate (i', j') by 2 Sxx_i'i Sigma_jj' mu.
//
// Sxx is addressed as Sxx[k * ldx + i] for the columns i of the tile's rows
// (the full matrix with ldx = p, or the column slab of a row group whose base
// pointer is offset by the group's first column).
__global__ __launch_bounds__(BLOCK) void theta_gs_kernel(
    const TileRect *__restrict__ rects, const int *__restrict__ active, int S,
    const double *__restrict__ partial, int64_t p, int64_t q, const double *__restrict__ Sxx,
    int64_t ldx, const double *__restrict__ Sxy, const double *__restrict__ Sigma,
    const double *__restrict__ GT, double *__restrict__ Theta, double lamT,
    double *__restrict__ dT, int *__restrict__ changed, unsigned long long *__restrict__ ctr,
    int esz) {
    const int e = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    if (!active[e]) {
        if (tid == 0) changed[e] = 0;
        return;
    }
    const TileRect rc = rects[e];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    __shared__ double Bs[TT][LDT];    // gradient snapshot, then corrected in place
    __shared__ double sxx[TT][LDT];   // Sxx[I, I]
    __shared__ double sig[TT][LDT];   // Sigma[J, J]
    const double *snap = partial + (int64_t)e * S * TT * TT;   // summed into part 0
    for (int k = tid; k < TT * TT; k += BLOCK) {
        const int r = k / TT, c = k % TT;
        Bs[r][c] = (r < R && c < C)
                       ? 2.0 * Sxy[(int64_t)(rc.r0 + r) * q + rc.c0 + c] + 2.0 * snap[k]
                       : 0.0;
        sxx[r][c] = (r < R && c < R) ? Sxx[(int64_t)(rc.r0 + r) * ldx + rc.r0 + c] : 0.0;
        sig[r][c] = (r < C && c < C) ? Sigma[(int64_t)(rc.c0 + r) * q + rc.c0 + c] : 0.0;
    }
    if (ctr && tid == 0) {
        const int64_t RC = (int64_t)R * C;
        atomicAdd(ctr + 0, 1ull);
        // snapshot: slabs Sxx[:, I] and V[:, J]
        atomicAdd(ctr + 1, (unsigned long long)(esz * p * (R + C)));
        atomicAdd(ctr + 2, (unsigned long long)(2 * RC * p));
        // Gauss-Seidel: Sxx[I, I], Sigma[J, J], Sxy / G / Theta reads, Theta and delta writes
        atomicAdd(ctr + 3, (unsigned long long)(8 * (R * R + C * C + 5 * RC)));
        atomicAdd(ctr + 4, (unsigned long long)(4 * RC * C));
    }
    __syncthreads();
    if (wid != 0) return;

    // Exact Gauss-Seidel by one wave: lane c owns column c of the tile.  Theta
    // and G of the next row are fetched while the current row is solved.
    const int c = lane;
    const bool colok = c < C;
    const double sjj = colok ? sig[c][c] : 1.0;
    double sigc[TT];                 // lane c keeps column c of Sigma[J, J]
#pragma unroll
    for (int l = 0; l < TT; ++l) sigc[l] = sig[l][c];
    int any_change = 0;
    double *dTe = dT + (int64_t)e * TT * TT;
    double th_n = 0.0, g_n = 0.0;
    auto fetch_row = [&](int r) {
        if (colok) {
            const int64_t ro = (int64_t)(rc.r0 + r) * q + rc.c0 + c;
            th_n = Theta[ro];
            g_n = GT[ro];
        }
    };
    fetch_row(0);
    for (int r = 0; r < R; ++r) {
        const double th0 = th_n;
        const double g = g_n;
        if (r + 1 < R) fetch_row(r + 1);
        const int64_t i = rc.r0 + r;
        double b = Bs[r][c];
        const double sii = sxx[r][r];
        const double a = 2.0 * sii * sjj, two_sii = 2.0 * sii;
        const bool act = colok && a > 0.0 && (fabs(g) > lamT || th0 != 0.0);
        const uint64_t mask = __ballot(act);
        const double ainv = act ? 1.0 / a : 0.0;
        const double thr = lamT * ainv;
        double w = 0.0, mu_mine = 0.0, th_new = th0;
        // Coordinate l (lane order): new value s = S_thr(Theta - b / a) from
        // lane l; every lane moves b by 2 Sxx_ii Sigma_lc (s - Theta_l).  The
        // chain from one coordinate's b to the next is b -> t -> clamp -> s ->
        // broadcast -> b.
        auto step = [&](int l, double sig_l) {
            const double x = two_sii * sig_l;
            const double th_l = readlane_f64(th0, l);
            const double t = th0 - b * ainv;
            const double st = t - fmax(fmin(t, thr), -thr);     // S_thr(t), exact zeros
            const double s_l = readlane_f64(st, l);
            const double mu = s_l - th_l;
            b = fma(s_l, x, fma(-th_l, x, b));
            w += sig_l * mu;
            if (c == l) {
                mu_mine = mu;
                th_new = s_l;
            }
        };
        if (__popcll(mask) >= GS_DENSE_ROW) {
#pragma unroll
            for (int l = 0; l < TT; ++l)
                if ((mask >> l) & 1ull) step(l, sigc[l]);
        } else {
            for (uint64_t m = mask; m; m &= m - 1) {
                const int l = __ffsll((unsigned long long)m) - 1;
                step(l, sig[l][c]);
            }
        }
        if (__ballot(mu_mine != 0.0)) any_change = 1;
        if (colok) {
            if (mu_mine != 0.0) Theta[i * q + rc.c0 + c] = th_new;
            dTe[r * TT + c] = mu_mine;
        }
        // later rows: b[r2][c] += 2 Sxx[r2][r] sum_l mu_l Sigma[l][c]
        // (lanes outside the tile add zeros: their sig entries are zero)
        const double w2 = 2.0 * w;
        for (int r2 = r + 1; r2 < R; r2 += 4) {
            double bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (r2 + u < R) bv[u] = Bs[r2 + u][c];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (r2 + u < R) Bs[r2 + u][c] = bv[u] + sxx[r2 + u][r] * w2;
        }
    }
    if (lane == 0) {
        changed[e] = any_change;
        // update (run only for a tile that changed): Sigma[J, :] read, V[I, :]
        // read and written
        if (ctr && any_change) {
            atomicAdd(ctr + 5, (unsigned long long)(esz * q * (C + 2 * R)));
            atomicAdd(ctr + 6, (unsigned long long)(2 * (int64_t)R * C * q));
        }
    }
}

// Out[m][n] += sum_k op(Delta)[m][k] S[k][n] for m < R, k < Kd and the
// columns [c_begin, c_end) of a row block (the maintained-product update of a
// tile).  op(Delta)[m][k] = Delta[m * TK + k], or Delta[k * TK + m] when
// `trans`.  Delta is staged in LDS once; each of the 4 waves owns 16 columns of
// every 64-column chunk, loads its S operands straight from global memory (one
// 128-byte row segment per k-step) and read-modify-writes Out from the MFMA
// accumulators.  All BLOCK threads call it.
// Instantiated with E = double; the mixed mode's FP32 rows use
// rowblock_update32.
template <int TR, int TK, class E>
__device__ void rowblock_update(const double *__restrict__ Delta, bool trans, int R, int Kd,
                                const E *__restrict__ S, int64_t lds,
                                E *__restrict__ Out, int64_t ldo, int64_t c_begin,
                                int64_t c_end, double (*dl)[TR + 2]) {
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    for (int e = tid; e < TK * TR; e += BLOCK) {
        const int k = e / TR, m = e % TR;
        dl[k][m] = (m < R && k < Kd) ? (trans ? Delta[k * TK + m] : Delta[m * TK + k]) : 0.0;
    }
    __syncthreads();
    constexpr int KST = TK / 4, NI = TR / 16, KH = KST / 2;
    const int col = lane & 15, krow = lane >> 4;
    // Per 64-column chunk: the current Out values go straight into the MFMA
    // accumulators, then the S operands stream in two halves of the K range.
#pragma unroll 1
    for (int64_t c0 = c_begin; c0 < c_end; c0 += 64) {
        const int64_t n = c0 + wid * 16 + col;
        const bool nv = n < c_end;
        v4d acc[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = i * 16 + krow + 4 * r;
                acc[i][r] = (nv && m < R) ? (double)Out[(int64_t)m * ldo + n] : 0.0;
            }
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            double bv[KH];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) {
                const int k = (h * KH + ks) * 4 + krow;
                bv[ks] = (nv && k < Kd) ? (double)S[(int64_t)k * lds + n] : 0.0;
            }
#pragma unroll
            for (int ks = 0; ks < KH; ++ks)
#pragma unroll
                for (int i = 0; i < NI; ++i)
                    acc[i] = mfma_f64_16x16x4(dl[(h * KH + ks) * 4 + krow][i * 16 + col], bv[ks],
                                              acc[i]);
        }
        if (nv) {
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = i * 16 + krow + 4 * r;
                    if (m < R) Out[(int64_t)m * ldo + n] = (E)acc[i][r];
                }
        }
    }
}


// rowblock_update from FP32 S and Out (row lengths multiples of 4, columns up
// to c_end, itself a multiple of 4): each wave owns 64 consecutive columns as
// 4 MFMA blocks j with the columns {4 c + j}, so a lane reads and writes four
// consecutive floats of a row; the S rows stream in groups of UPD32_GROUP
// k-steps whose loads are all issued before their products; FP32
// accumulation.  Every load is unconditional, from a row and column clamped
// into the valid range (R, Kd >= 1; c_end - 4 >= c_begin), so that a chunk's
// loads are all in flight together: lanes past c_end and rows past R compute
// values that are never stored, and S rows past Kd are replaced by zeros.
// All BLOCK threads call it.
constexpr int UPD32_GROUP = 8;
template <int TR, int TK>
__device__ void rowblock_update32(const double *__restrict__ Delta, bool trans, int R, int Kd,
                                  const float *__restrict__ S, int64_t lds,
                                  float *__restrict__ Out, int64_t ldo, int64_t c_begin,
                                  int64_t c_end, float (*dl)[TR + 4]) {
    static_assert(TR == 64 && TK == 64, "one 64 x 64 delta per tile");
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    for (int e = tid; e < TK * TR; e += BLOCK) {
        const int k = e / TR, m = e % TR;
        dl[k][m] = (m < R && k < Kd) ? (float)(trans ? Delta[k * TK + m] : Delta[m * TK + k])
                                     : 0.f;
    }
    __syncthreads();
    const int col = lane & 15, krow = lane >> 4;
#pragma unroll 1
    for (int64_t c0 = c_begin + wid * 64; c0 < c_end; c0 += 4 * 64) {
        const int64_t n = c0 + 4 * col;              // this lane's four columns
        const bool nv = n < c_end;
        const int64_t nc = nv ? n : c_end - 4;       // in-bounds column for every lane
        f32x4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = i * 16 + 4 * krow + r;
                const f32x4 v = *reinterpret_cast<const f32x4 *>(
                    Out + (int64_t)(m < R ? m : R - 1) * ldo + nc);
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j][r] = v[j];
            }
#pragma unroll 1
        for (int h = 0; h < TK / 4 / UPD32_GROUP; ++h) {
            f32x4 bvs[UPD32_GROUP];
#pragma unroll
            for (int u = 0; u < UPD32_GROUP; ++u) {
                const int k = (h * UPD32_GROUP + u) * 4 + krow;
                const f32x4 v =
                    *reinterpret_cast<const f32x4 *>(S + (int64_t)(k < Kd ? k : Kd - 1) * lds + nc);
                bvs[u] = k < Kd ? v : f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < UPD32_GROUP; ++u) {
                const int k = (h * UPD32_GROUP + u) * 4 + krow;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float av = dl[k][i * 16 + col];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = mfma_f32_16x16x4(av, bvs[u][j], acc[i][j]);
                }
            }
        }
        if (nv) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = i * 16 + 4 * krow + r;
                    if (m < R)
                        *reinterpret_cast<f32x4 *>(Out + (int64_t)m * ldo + n) =
                            f32x4{acc[i][0][r], acc[i][1][r], acc[i][2][r], acc[i][3][r]};
                }
        }
    }
}

constexpr int UPD_CHUNKS = 4;   // 64-column chunks per update workgroup
constexpr int UPD_MINB = 4;     // workgroups per CU the update kernels are built for

// V[I, :] += dTheta[I, J] Sigma[J, :] for every changed tile of the wave.
template <class E>
__global__ __launch_bounds__(BLOCK, UPD_MINB) void theta_v_update_kernel(
    const TileRect *__restrict__ rects, int64_t q, const E *__restrict__ Sigma,
    const double *__restrict__ dT, const int *__restrict__ changed, E *__restrict__ V) {
    const int e = blockIdx.y;
    if (!changed[e]) return;
    const TileRect rc = rects[e];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int64_t c_begin = (int64_t)blockIdx.x * 64 * UPD_CHUNKS;
    const int64_t c_end = std::min<int64_t>(q, c_begin + 64 * UPD_CHUNKS);
    __shared__ double dl[TT][TT + 2];
    rowblock_update<TT, TT, E>(dT + (int64_t)e * TT * TT, false, R, C,
                               Sigma + (int64_t)rc.c0 * q, q, V + (int64_t)rc.r0 * q, q, c_begin,
                               c_end, dl);
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
// A 64 x 64 block of doubles in LDS with an XOR swizzle: element (r, c) sits
// at r * 64 + (c ^ r), so a row (fixed r, lane c) and a column (fixed c, lane r)
// of the block both touch 64 distinct slots.
struct Swz64 {
    double *p;
    __device__ __forceinline__ double &operator()(int r, int c) const {
        return p[r * 64 + (c ^ r)];
    }
};
// The same block unswizzled, for one that is only written and read by rows
// (lane = column): the slot of (r, c) is then an immediate offset plus the
// lane's.
struct Row64 {
    double *p;
    __device__ __forceinline__ double &operator()(int r, int c) const { return p[r * 64 + c]; }
};

// Exact Gauss-Seidel over the active coordinates of one tile, row by row,
// lane = column: the row's coordinates in lane order with v_readlane
// broadcasts, the dependent chain of one step three fused multiply-adds and
// a clamp (soft threshold as t - max(min(t, hi), lo)), then the moves of the
// row folded into the later rows.  A tile with fewer than GS_WIDE_MIN active
// coordinates is run by one wavefront, which forms each coupling x_l(c) in
// the step and folds each row into all later rows itself.  A denser tile
// is run by the four wavefronts of the workgroup with one workgroup barrier
// per row r:
//   wave 0 runs only the coordinate chain of row r, the couplings read from
//     LDS a step ahead; it writes D, the tile's delta, and the row's moves
//     and w1, w4 sums for the other waves, and after the barrier folds row
//     r's moves into row r + 1;
//   wave 1 forms the couplings of row r + 1 (from the Sigma / Psi rows of the
//     tile, the (J, J) columns held in registers) into the other of two LDS
//     buffers;
//   waves 2 and 3 fold row r - 1's moves into rows r + 1 .. R - 1 (even and
//     odd rows), holding the rows of S_IJ and SP_IJ in registers.
// So the chain of row r + 1 starts right after the barrier that ends row r,
// with its couplings formed and every earlier row's moves folded in, in row
// order.  Both forms compute every value as one wavefront doing all of it
// would, except the four-wave form's sums w2, w3 of row r + 1 (a butterfly
// sum instead of four strided partial sums).
constexpr int GS_WIDE_MIN = 256;

// The one-wavefront form of lambda_gs_kernel for a sparse tile: wave 0 of the
// workgroup after the snapshot, S_IJ and P_IJ are staged (Bs, St, Pt).
__device__ __forceinline__ void lambda_gs_one_wave(
    const TileRect rc, int e, int64_t q, const double *__restrict__ Sigma,
    const double *__restrict__ Psi, const double *__restrict__ GL,
    const double *__restrict__ Lam, double lamL, double *__restrict__ D,
    double *__restrict__ dD, int *__restrict__ changed, unsigned long long *__restrict__ ctr,
    int esz, const Swz64 Bs, const Swz64 St, const Swz64 Pt) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const bool diag = rc.r0 == rc.c0;
    const int c = lane;
    const bool inC = c < C;
    const double s_jj = inC ? Sigma[(int64_t)(rc.c0 + c) * q + rc.c0 + c] : 0.0;
    const double p_jj = inC ? Psi[(int64_t)(rc.c0 + c) * q + rc.c0 + c] : 0.0;
    // lane c keeps column c of the (J, J) blocks in registers for the whole
    // tile
    double sJc[T], pJc[T];
#pragma unroll
    for (int l = 0; l < T; ++l) {
        const int64_t o = (int64_t)(rc.c0 + l) * q + rc.c0 + c;
        sJc[l] = (inC && l < C) ? Sigma[o] : 0.0;
        pJc[l] = (inC && l < C) ? Psi[o] : 0.0;
    }
    int any_change = 0;
    double *dDe = dD + (int64_t)e * T * T;
    // Per-row global operands, fetched one row ahead: lane r2 holds
    // Sigma_II[r][r2] and Psi_II[r][r2]; lane c holds Lambda, D and G at (r, c).
    // (The prefetch of D's next row precedes this row's writes: the only
    // writes into later rows of the tile are the mirror entries of a diagonal
    // tile, below the diagonal, which the coordinate loop never reads.)
    const bool inR = lane < R;
    double srow_n = 0.0, prow_n = 0.0, lam_n = 0.0, d_n = 0.0, g_n = 0.0;
    auto fetch_row = [&](int r) {
        const int64_t ro = (int64_t)(rc.r0 + r) * q;
        if (inR) {
            srow_n = Sigma[ro + rc.r0 + lane];
            prow_n = Psi[ro + rc.r0 + lane];
        }
        if (inC) {
            lam_n = Lam[ro + rc.c0 + c];
            d_n = D[ro + rc.c0 + c];
            g_n = GL[ro + rc.c0 + c];
        }
    };
    fetch_row(0);
    for (int r = 0; r < R; ++r) {
        const double srow = srow_n, prow = prow_n, lamv = lam_n, d0 = d_n, g = g_n;
        if (r + 1 < R) fetch_row(r + 1);
        const int64_t i = rc.r0 + r;
        const bool colok = inC && (!diag || c >= r);
        const double s_ij = St(r, c), p_ij = Pt(r, c);
        double b = Bs(r, c);
        const double sii = readlane_f64(srow, r), pii = readlane_f64(prow, r);
        const double spii = sii + pii;
        const bool self = diag && c == r;
        const double a = self ? sii * sii + 2.0 * sii * pii
                              : s_ij * s_ij + sii * s_jj + sii * p_jj + s_jj * pii +
                                    2.0 * s_ij * p_ij;
        const bool act = colok && a > 0.0 && (fabs(g) > lamL || lamv != 0.0);
        const uint64_t mask = __ballot(act);
        const double ainv = act ? 1.0 / a : 0.0;
        const double thr = lamL * ainv;
        // c = Lambda_ij + D_ij with D_ij as left by earlier passes (zero on the
        // first), unchanged until the coordinate is visited
        const double cv = lamv + d0;
        double w1 = 0.0, w4 = 0.0, mu_mine = 0.0, s_mine;
        // Coordinate l of the row (lane order): its new value is
        // s = S_thr(cv - b / a), broadcast from lane l; every lane then moves
        // b by mu_e x_l with mu = s - cv_l.  The chain from one coordinate's b
        // to the next is b -> t -> clamp -> s -> broadcast -> b; the coupling
        // x_l and the cv_l term do not depend on b.  A diagonal tile halves
        // the move of its self coordinate (l == r).
        // One coordinate step; the (J, J) column entries come from registers
        // (an unrolled scan over the row, masked by the active lanes).
        const double sp_ij = s_ij + p_ij;
        const double thr_hi = __builtin_canonicalize(thr), thr_lo = __builtin_canonicalize(-thr);
        auto step = [&](int l, double sJl, double pJl, auto diag_tile) {
            constexpr bool DIAG = decltype(diag_tile)::value;
            const double s_il = readlane_f64(s_ij, l), p_il = readlane_f64(p_ij, l);
            const double cv_l = readlane_f64(cv, l);
            // x = SP_ii S_lc + SP_il S_ic + P_ic S_il + P_lc S_ii
            const double x = fma(spii, sJl, fma(sii, pJl, fma(s_il, sp_ij, p_il * s_ij)));
            const double t = cv - b * ainv;
            const double st = t - fmax(fmin(t, thr_hi), thr_lo);   // S_thr(t), exact zeros
            const double s_l = readlane_f64(st, l);
            const double mu = s_l - cv_l;
            double mue = mu;
            if (DIAG && l == r) {
                mue = 0.5 * mu;
                b += mue * x;
            } else {
                b = fma(s_l, x, fma(-cv_l, x, b));
            }
            w1 += mue * sJl;
            w4 += mue * pJl;
            s_mine = (c == l) ? st : s_mine;
        };
        auto row_dense = [&](auto diag_tile) {
#pragma unroll
            for (int l = 0; l < T; ++l)
                if ((mask >> l) & 1ull) step(l, sJc[l], pJc[l], diag_tile);
        };
        s_mine = cv;                         // unvisited lanes keep their value
        if (mask) {
            if (diag)
                row_dense(std::integral_constant<bool, true>{});
            else
                row_dense(std::integral_constant<bool, false>{});
        }
        mu_mine = ((mask >> c) & 1ull) ? s_mine - cv : 0.0;
        if (colok && mu_mine != 0.0) {
            // new D = S - Lambda, so a thresholded coordinate gives exactly
            // Lambda + D = 0
            D[i * q + rc.c0 + c] = s_mine - lamv;
            D[(int64_t)(rc.c0 + c) * q + i] = s_mine - lamv;
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
        //   b[r2][c] += SP_II[r2][r] w1_c + S_IJ[r][c] w2_r2 + P_IJ[r][c] w3_r2
        //               + S_II[r][r2] w4_c,
        //   w2_r2 = sum_l SP_IJ[r2][l] mu_e,l,   w3_r2 = sum_l S_IJ[r2][l] mu_e,l.
        const double mue_mine = (diag && c == r) ? 0.5 * mu_mine : mu_mine;
        uint64_t moved = __ballot(mu_mine != 0.0);
        if (moved == 0) continue;
        any_change = 1;
        double w2 = 0.0, w3 = 0.0;            // lane r2 accumulates row r2's values
        if (__popcll(moved) >= 16) {
            // dense row: all 64 columns, four partial sums, loads in flight
            double a2[4] = {0.0, 0.0, 0.0, 0.0}, a3[4] = {0.0, 0.0, 0.0, 0.0};
            for (int l0 = 0; l0 < T; l0 += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double m = readlane_f64(mue_mine, l0 + u);
                    const double sv = St(lane, l0 + u);
                    a2[u] += (sv + Pt(lane, l0 + u)) * m;
                    a3[u] += sv * m;
                }
            }
            w2 = (a2[0] + a2[1]) + (a2[2] + a2[3]);
            w3 = (a3[0] + a3[1]) + (a3[2] + a3[3]);
        } else {
            while (moved) {
                const int l = __ffsll((unsigned long long)moved) - 1;
                moved &= moved - 1;
                const double m = readlane_f64(mue_mine, l);
                const double sv = St(lane, l);
                w2 += (sv + Pt(lane, l)) * m;
                w3 += sv * m;
            }
        }
        // (lanes outside the tile add zeros: their LDS entries are zero)
        for (int r2 = r + 1; r2 < R; r2 += 4) {
            double bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (r2 + u < R) bv[u] = Bs(r2 + u, c);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (r2 + u < R) {
                    const int rr = r2 + u;
                    const double w2r = readlane_f64(w2, rr), w3r = readlane_f64(w3, rr);
                    const double s_r2 = readlane_f64(srow, rr), p_r2 = readlane_f64(prow, rr);
                    Bs(rr, c) = bv[u] + ((s_r2 + p_r2) * w1 + s_ij * w2r + p_ij * w3r + s_r2 * w4);
                }
            }
        }
    }
    if (lane == 0) {
        changed[e] = any_change;
        // update (run only for a tile that changed): Sigma rows read, U rows
        // read and written (both index sets of an off-diagonal tile)
        if (ctr && any_change) {
            const int64_t ub = diag ? esz * q * 3 * R : esz * q * 3 * (R + C);
            atomicAdd(ctr + 5, (unsigned long long)ub);
            atomicAdd(ctr + 6, (unsigned long long)((diag ? 2 : 4) * (int64_t)R * C * q));
        }
    }
}


__global__ __launch_bounds__(BLOCK) void lambda_gs_kernel(
    const TileRect *__restrict__ rects, const int *__restrict__ active, int S,
    const double *__restrict__ partial, int64_t q, const double *__restrict__ Sigma,
    const double *__restrict__ Psi, const double *__restrict__ GL,
    const double *__restrict__ Lam, double lamL, double *__restrict__ D,
    double *__restrict__ dD, int *__restrict__ changed, unsigned long long *__restrict__ ctr,
    int esz) {
    static_assert(T == 64 && BLOCK == 4 * WAVE, "one 64-wide tile, four wavefronts");
    const int e = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wid = __builtin_amdgcn_readfirstlane(tid / WAVE);
    if (!active[e]) {
        if (tid == 0) changed[e] = 0;
        return;
    }
    const TileRect rc = rects[e];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const bool diag = rc.r0 == rc.c0;
    // LDS: the b snapshot, S_IJ and P_IJ (XOR-swizzled: rows and columns are
    // both conflict-free); in the four-wave form, once waves 2 and 3 hold
    // their rows of S_IJ and SP_IJ, the two coupling blocks X (l, c) take the
    // place of S_IJ and P_IJ, row r of the snapshot carries row r's moves once
    // its chain has read it, and the w1 / w4 sums of the last two rows and
    // their "row moved" flags follow.
    __shared__ double lds[3 * T * T + 4 * T + 2];
    const Swz64 Bs{lds}, St{lds + T * T}, Pt{lds + 2 * T * T};
    const Row64 X0{lds + T * T}, X1{lds + 2 * T * T};
    double *const W1 = lds + 3 * T * T, *const W4 = W1 + 2 * T;
    int *const MOV = reinterpret_cast<int *>(W4 + 2 * T);
    const double *snap = partial + (int64_t)e * S * T * T;    // summed into part 0
    for (int k = tid; k < T * T; k += BLOCK) {
        const int r = k / T, c = k % T;
        const bool ij = r < R && c < C;
        const int64_t o = (int64_t)(rc.r0 + r) * q + rc.c0 + c;
        Bs(r, c) = ij ? snap[k] + GL[o] : 0.0;
        St(r, c) = ij ? Sigma[o] : 0.0;
        Pt(r, c) = ij ? Psi[o] : 0.0;
    }
    if (ctr && tid == 0) {
        const int64_t RC = (int64_t)R * C;
        atomicAdd(ctr + 0, 1ull);
        // snapshot: slabs SP[:, I], U[:, J], U[:, I], Psi[:, J]
        atomicAdd(ctr + 1, (unsigned long long)(esz * 2 * q * (R + C)));
        atomicAdd(ctr + 2, (unsigned long long)(4 * RC * q));
        // Gauss-Seidel: six Sigma / Psi blocks, G and Lambda reads, D (both
        // triangles) and delta writes
        atomicAdd(ctr + 3, (unsigned long long)(8 * (2 * R * R + 2 * C * C + 7 * RC)));
        atomicAdd(ctr + 4, (unsigned long long)(16 * RC * C));
    }
    __syncthreads();
    if (active[e] < GS_WIDE_MIN) {
        if (wid == 0)
            lambda_gs_one_wave(rc, e, q, Sigma, Psi, GL, Lam, lamL, D, dD, changed, ctr, esz, Bs,
                               St, Pt);
        return;
    }
    // Waves 0, 1: column `lane` of S_JJ and P_JJ; waves 2, 3: row `lane` of
    // S_IJ and SP_IJ (zero outside the tile).
    double regA[T], regB[T];
    if (wid >= 2) {
#pragma unroll
        for (int l = 0; l < T; ++l) {
            const double s = St(lane, l);
            regA[l] = s;
            regB[l] = s + Pt(lane, l);
        }
    } else {
        const bool inC = lane < C;
#pragma unroll
        for (int l = 0; l < T; ++l) {
            const int64_t o = (int64_t)(rc.c0 + l) * q + rc.c0 + lane;
            regA[l] = (inC && l < C) ? Sigma[o] : 0.0;
            regB[l] = (inC && l < C) ? Psi[o] : 0.0;
        }
    }
    __syncthreads();                                  // the staging buffers are free
    // x_l(c) = SP_ii S_lc + S_ii P_lc + S_il SP_ic + P_il S_ic of row rn
    auto couplings = [&](int rn, const Row64 &X) {
        const int64_t ro = (int64_t)(rc.r0 + rn) * q;
        const double sii = Sigma[ro + rc.r0 + rn], pii = Psi[ro + rc.r0 + rn];
        const bool inC = lane < C;
        const double s_c = inC ? Sigma[ro + rc.c0 + lane] : 0.0;
        const double p_c = inC ? Psi[ro + rc.c0 + lane] : 0.0;
        const double spii = sii + pii, sp_c = s_c + p_c;
#pragma unroll
        for (int l = 0; l < T; ++l) {
            const double s_il = readlane_f64(s_c, l), p_il = readlane_f64(p_c, l);
            X(l, lane) = fma(spii, regA[l], fma(sii, regB[l], fma(s_il, sp_c, p_il * s_c)));
        }
    };
    if (wid == 1) couplings(0, X0);
    __syncthreads();

    // ---- per-row state of wave 0 (coordinate chain) ----
    const int c = lane;
    const bool inC = c < C, inR = lane < R;
    const double s_jj = (wid == 0 && inC) ? Sigma[(int64_t)(rc.c0 + c) * q + rc.c0 + c] : 0.0;
    const double p_jj = (wid == 0 && inC) ? Psi[(int64_t)(rc.c0 + c) * q + rc.c0 + c] : 0.0;
    int any_change = 0;
    double *dDe = dD + (int64_t)e * T * T;
    // Row operands fetched one row ahead: lane r2 holds Sigma_II[r][r2] and
    // Psi_II[r][r2]; lane c holds S_IJ, P_IJ, Lambda, D and G at (r, c).
    // (The prefetch of D's next row precedes this row's writes: the only
    // writes into later rows of the tile are the mirror entries of a diagonal
    // tile, below the diagonal, which the coordinate loop never reads.)
    double srow_n = 0.0, prow_n = 0.0, sij_n = 0.0, pij_n = 0.0;
    double lam_n = 0.0, d_n = 0.0, g_n = 0.0;
    auto fetch_row = [&](int r) {
        const int64_t ro = (int64_t)(rc.r0 + r) * q;
        srow_n = inR ? Sigma[ro + rc.r0 + lane] : 0.0;
        prow_n = inR ? Psi[ro + rc.r0 + lane] : 0.0;
        sij_n = inC ? Sigma[ro + rc.c0 + c] : 0.0;
        pij_n = inC ? Psi[ro + rc.c0 + c] : 0.0;
        if (wid == 0 && inC) {
            lam_n = Lam[ro + rc.c0 + c];
            d_n = D[ro + rc.c0 + c];
            g_n = GL[ro + rc.c0 + c];
        }
    };
    if (wid == 0 || wid >= 2) fetch_row(0);

    for (int r = 0; r < R; ++r) {
        const int par = r & 1;
        // the row operands of row r (waves 2, 3 use those of row r - 1,
        // fetched in the previous iteration)
        const double srow = srow_n, prow = prow_n, s_ij = sij_n, p_ij = pij_n;
        // wave 0's results of the row, used after the barrier
        double w1 = 0.0, w4 = 0.0, mue_mine = 0.0;
        uint64_t moved = 0;
        if (wid == 0) {
            const double lamv = lam_n, d0 = d_n, g = g_n;
            if (r + 1 < R) fetch_row(r + 1);
            const Row64 X = par ? X1 : X0;
            const int64_t i = rc.r0 + r;
            const bool colok = inC && (!diag || c >= r);
            double b = Bs(r, c);
            const double sii = readlane_f64(srow, r), pii = readlane_f64(prow, r);
            const bool self = diag && c == r;
            const double a = self ? sii * sii + 2.0 * sii * pii
                                  : s_ij * s_ij + sii * s_jj + sii * p_jj + s_jj * pii +
                                        2.0 * s_ij * p_ij;
            const bool act = colok && a > 0.0 && (fabs(g) > lamL || lamv != 0.0);
            const uint64_t mask = __ballot(act);
            const double ainv = act ? 1.0 / a : 0.0;
            const double thr = lamL * ainv;
            // c = Lambda_ij + D_ij with D_ij as left by earlier passes (zero
            // on the first), unchanged until the coordinate is visited
            const double cv = lamv + d0;
            double s_mine = cv;                      // unvisited lanes keep their value
            const double thr_hi = __builtin_canonicalize(thr), thr_lo = __builtin_canonicalize(-thr);
            // Coordinate l of the row (lane order): its new value is
            // s = S_thr(cv - b / a), broadcast from lane l; every lane then
            // moves b by mu_e x_l with mu = s - cv_l.  The chain from one
            // coordinate's b to the next is b -> t -> clamp -> s -> broadcast
            // -> b; x_l and cv_l do not depend on b.  A diagonal tile halves
            // the move of its self coordinate (l == r).
            auto step = [&](int l, double x, auto diag_tile) {
                constexpr bool DIAG = decltype(diag_tile)::value;
                const double cv_l = readlane_f64(cv, l);
                const double t = cv - b * ainv;
                const double st = t - fmax(fmin(t, thr_hi), thr_lo);   // S_thr(t), exact zeros
                const double s_l = readlane_f64(st, l);
                const double mu = s_l - cv_l;
                double mue = mu;
                if (DIAG && l == r) {
                    mue = 0.5 * mu;
                    b += mue * x;
                } else {
                    b = fma(s_l, x, fma(-cv_l, x, b));
                }
                w1 += mue * regA[l];
                w4 += mue * regB[l];
                s_mine = (c == l) ? st : s_mine;
            };
            auto row = [&](auto diag_tile) {
                double xn = X(0, c);             // the next coupling, read one step ahead
#pragma unroll
                for (int l = 0; l < T; ++l) {
                    const double x = xn;
                    if (l + 1 < T) xn = X(l + 1, c);
                    if ((mask >> l) & 1ull) step(l, x, diag_tile);
                }
            };
            if (mask) {
                if (diag)
                    row(std::integral_constant<bool, true>{});
                else
                    row(std::integral_constant<bool, false>{});
            }
            const double mu_mine = ((mask >> c) & 1ull) ? s_mine - cv : 0.0;
            if (colok && mu_mine != 0.0) {
                // new D = S - Lambda, so a thresholded coordinate gives
                // exactly Lambda + D = 0
                D[i * q + rc.c0 + c] = s_mine - lamv;
                D[(int64_t)(rc.c0 + c) * q + i] = s_mine - lamv;
            }
            if (inC) {
                if (!diag) {
                    dDe[r * T + c] = mu_mine;
                } else if (c >= r) {                 // symmetric delta of a diagonal tile
                    dDe[r * T + c] = mu_mine;
                    dDe[c * T + r] = mu_mine;
                }
            }
            mue_mine = (diag && c == r) ? 0.5 * mu_mine : mu_mine;
            moved = __ballot(mu_mine != 0.0);
            if (moved) any_change = 1;
            // Later rows r2 of the tile then gain
            //   b[r2][c] += SP_II[r2][r] w1_c + S_IJ[r][c] w2_r2 + P_IJ[r][c] w3_r2
            //               + S_II[r][r2] w4_c,
            //   w2_r2 = sum_l SP_IJ[r2][l] mu_e,l,   w3_r2 = sum_l S_IJ[r2][l] mu_e,l.
            Bs(r, c) = mue_mine;
            W1[par * T + c] = w1;
            W4[par * T + c] = w4;
            if (lane == 0) MOV[par] = moved != 0;
        } else if (wid == 1) {
            if (r + 1 < R) couplings(r + 1, par ? X0 : X1);
        } else {
            // fold the moves of row src = r - 1 into rows src + 2 .. R - 1
            // (this wave's parity of them); fetch row r's operands for the
            // next row
            const int src = r - 1;
            if (r + 1 < R) fetch_row(r);
            if (src >= 0 && MOV[src & 1] && src + 2 < R) {
                const double m_l = Bs(src, lane);     // lane l: mu_e of coordinate (src, l)
                double a2[4] = {0.0, 0.0, 0.0, 0.0}, a3[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int l0 = 0; l0 < T; l0 += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double m = readlane_f64(m_l, l0 + u);
                        a2[u] += regB[l0 + u] * m;
                        a3[u] += regA[l0 + u] * m;
                    }
                }
                const double w2 = (a2[0] + a2[1]) + (a2[2] + a2[3]);   // lane r2: row r2's sums
                const double w3 = (a3[0] + a3[1]) + (a3[2] + a3[3]);
                const double w1s = W1[(src & 1) * T + lane], w4s = W4[(src & 1) * T + lane];
                int rr = src + 2;
                if ((rr & 1) != (wid & 1)) ++rr;
                for (; rr < R; rr += 2) {
                    const double w2r = readlane_f64(w2, rr), w3r = readlane_f64(w3, rr);
                    const double s_r2 = readlane_f64(srow, rr), p_r2 = readlane_f64(prow, rr);
                    Bs(rr, c) = Bs(rr, c) + ((s_r2 + p_r2) * w1s + s_ij * w2r + p_ij * w3r +
                                             s_r2 * w4s);
                }
            }
        }
        __syncthreads();
        if (wid == 0 && moved && r + 1 < R) {
            // row r + 1 now, the rows after it by waves 2 and 3 during the next row
            const double w2n = wave_sum((sij_n + pij_n) * mue_mine);
            const double w3n = wave_sum(sij_n * mue_mine);
            const double s_r2 = readlane_f64(srow, r + 1), p_r2 = readlane_f64(prow, r + 1);
            Bs(r + 1, c) =
                Bs(r + 1, c) + ((s_r2 + p_r2) * w1 + s_ij * w2n + p_ij * w3n + s_r2 * w4);
        }
    }
    if (wid == 0 && lane == 0) {
        changed[e] = any_change;
        // update (run only for a tile that changed): Sigma rows read, U rows
        // read and written (both index sets of an off-diagonal tile)
        if (ctr && any_change) {
            const int64_t ub = diag ? esz * q * 3 * R : esz * q * 3 * (R + C);
            atomicAdd(ctr + 5, (unsigned long long)ub);
            atomicAdd(ctr + 6, (unsigned long long)((diag ? 2 : 4) * (int64_t)R * C * q));
        }
    }
}

// U[I, :] += dD Sigma[J, :] and U[J, :] += dD^T Sigma[I, :] (off-diagonal
// tiles), or U[I, :] += dD_sym Sigma[I, :] (diagonal tiles).
template <class E>
__global__ __launch_bounds__(BLOCK, UPD_MINB) void lambda_u_update_kernel(
    const TileRect *__restrict__ rects, int64_t q, const E *__restrict__ Sigma,
    const double *__restrict__ dD, const int *__restrict__ changed, E *__restrict__ U) {
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
        rowblock_update<T, T, E>(dDe, false, R, C, Sigma + (int64_t)rc.c0 * q, q,
                                 U + (int64_t)rc.r0 * q, q, c_begin, c_end, dl);
    else
        rowblock_update<T, T, E>(dDe, true, C, R, Sigma + (int64_t)rc.r0 * q, q,
                                 U + (int64_t)rc.c0 * q, q, c_begin, c_end, dl);
}

// The updates on FP32 copies (row length ld): V32[I, :] += dTheta Sigma32[J, :];
// U32 as lambda_u_update_kernel.  UPD32_COLS columns per workgroup; built for
// three workgroups per CU (the register budget of the eight-k-step groups).
constexpr int UPD32_COLS = 1024, UPD32_MINB = 3;
__global__ __launch_bounds__(BLOCK, UPD32_MINB) void theta_v_update32_kernel(
    const TileRect *__restrict__ rects, int64_t ld, const float *__restrict__ Sigma,
    const double *__restrict__ dT, const int *__restrict__ changed, float *__restrict__ V) {
    const int e = blockIdx.y;
    if (!changed[e]) return;
    const TileRect rc = rects[e];
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int64_t c_begin = (int64_t)blockIdx.x * UPD32_COLS;
    const int64_t c_end = std::min<int64_t>(ld, c_begin + UPD32_COLS);
    __shared__ float dl[TT][TT + 4];
    rowblock_update32<TT, TT>(dT + (int64_t)e * TT * TT, false, R, C, Sigma + (int64_t)rc.c0 * ld,
                              ld, V + (int64_t)rc.r0 * ld, ld, c_begin, c_end, dl);
}

__global__ __launch_bounds__(BLOCK, UPD32_MINB) void lambda_u_update32_kernel(
    const TileRect *__restrict__ rects, int64_t ld, const float *__restrict__ Sigma,
    const double *__restrict__ dD, const int *__restrict__ changed, float *__restrict__ U) {
    const int e = blockIdx.y, half = blockIdx.z;
    if (!changed[e]) return;
    const TileRect rc = rects[e];
    const bool diag = rc.r0 == rc.c0;
    if (diag && half == 1) return;
    const int R = rc.r1 - rc.r0, C = rc.c1 - rc.c0;
    const int64_t c_begin = (int64_t)blockIdx.x * UPD32_COLS;
    const int64_t c_end = std::min<int64_t>(ld, c_begin + UPD32_COLS);
    __shared__ float dl[T][T + 4];
    const double *dDe = dD + (int64_t)e * T * T;
    if (half == 0)
        rowblock_update32<T, T>(dDe, false, R, C, Sigma + (int64_t)rc.c0 * ld, ld,
                                U + (int64_t)rc.r0 * ld, ld, c_begin, c_end, dl);
    else
        rowblock_update32<T, T>(dDe, true, C, R, Sigma + (int64_t)rc.r0 * ld, ld,
                                U + (int64_t)rc.c0 * ld, ld, c_begin, c_end, dl);
}

// Parts of the K range per tile snapshot: enough wavefronts per launch
// (about SNAP_WAVES) to fill the GPU, at least SNAP_MIN_ROWS rows per part, at
// most CD_MAX_PARTS parts.
constexpr int64_t SNAP_WAVES = 8192, SNAP_MIN_ROWS = 256;
int snapshot_parts(int nrect, int quadrants, int64_t K) {
    int64_t S = SNAP_WAVES / std::max<int64_t>(1, (int64_t)nrect * quadrants);
    S = std::min<int64_t>(S, K / SNAP_MIN_ROWS);
    return (int)std::max<int64_t>(1, std::min<int64_t>(CD_MAX_PARTS, S));
}

inline void record(hipStream_t s, const WaveProbe *probe, int k) {
    if (probe) CGGM_HIP(hipEventRecord(probe->ev[k], s));
}

}  // namespace

void theta_activity(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t q,
                    const double *GT, const double *Theta, double lamT, int *active) {
    if (nrect <= 0) return;
    tile_activity_kernel<<<nrect, BLOCK, 0, s>>>(rects_dev, q, GT, Theta, lamT, 0, active);
    CGGM_LAUNCH_CHECK();
}

void lambda_activity(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t q,
                     const double *GL, const double *Lam, double lamL, int *active) {
    if (nrect <= 0) return;
    tile_activity_kernel<<<nrect, BLOCK, 0, s>>>(rects_dev, q, GL, Lam, lamL, 1, active);
    CGGM_LAUNCH_CHECK();
}

void theta_wave(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                int64_t p, int64_t q, const double *Sxx, int64_t ldx, const double *Sxy,
                const double *Sigma, double *V, const double *GT, double *Theta, double lamT,
                double *dT, int *changed, const CdScratch &scr, const WaveProbe *probe,
                const SweepF32 *f32) {
    if (nrect <= 0) return;
    constexpr int NB = snap_blocks_per_tile<TT>();
    const int S = snapshot_parts(nrect, NB, p);
    const bool lo = f32 && f32->on;
    record(s, probe, 0);
    const int full = f32 ? f32->full_rects : -1;
    if (lo) {
        SnapArgs<1, float> args{{f32->Sxx}, {f32->ldx}, {f32->V}, {f32->ldq}};
        snapshot<TT, 1, float>(s, rects_dev, active, S, nrect, p, args, full, scr.partial);
    } else {
        SnapArgs<1, double> args{{Sxx}, {ldx}, {V}, {q}};
        snapshot<TT, 1, double>(s, rects_dev, active, S, nrect, p, args, full, scr.partial);
    }
    sum_snapshots<TT>(s, active, nrect, S, scr.partial);
    record(s, probe, 1);
    theta_gs_kernel<<<nrect, BLOCK, 0, s>>>(rects_dev, active, S, scr.partial, p, q, Sxx, ldx,
                                            Sxy,
                                            Sigma, GT, Theta, lamT, dT, changed,
                                            probe ? probe->counters : nullptr,
                                            lo ? (int)sizeof(float) : (int)sizeof(double));
    CGGM_LAUNCH_CHECK();
    record(s, probe, 2);
    const int64_t cols_per_wg = 64 * UPD_CHUNKS;
    if (lo) {
        dim3 grid((unsigned)((f32->ldq + UPD32_COLS - 1) / UPD32_COLS), (unsigned)nrect);
        theta_v_update32_kernel<<<grid, BLOCK, 0, s>>>(rects_dev, f32->ldq, f32->Sigma, dT,
                                                       changed, f32->V);
    } else {
        dim3 grid((unsigned)((q + cols_per_wg - 1) / cols_per_wg), (unsigned)nrect);
        theta_v_update_kernel<double><<<grid, BLOCK, 0, s>>>(rects_dev, q, Sigma, dT, changed, V);
    }
    CGGM_LAUNCH_CHECK();
    record(s, probe, 3);
}

// b snapshot: G + (SP U)[I, J] + ((Psi U)[J, I])^T
//   = G + SP[:, I]^T U[:, J] + U[:, I]^T Psi[:, J]   (SP, Psi symmetric)
int lambda_snapshot(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                    int64_t q, const double *SP, const double *U, const double *Psi,
                    const CdScratch &scr, int full) {
    if (nrect <= 0) return 0;
    constexpr int NB = snap_blocks_per_tile<T>();
    const int S = snapshot_parts(nrect, NB, q);
    SnapArgs<2, double> args{{SP, U}, {q, q}, {U, Psi}, {q, q}};
    snapshot<T, 2, double>(s, rects_dev, active, S, nrect, q, args, full, scr.partial);
    sum_snapshots<T>(s, active, nrect, S, scr.partial);
    return S;
}

int lambda_snapshot(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                    int64_t q, const float *SP, const float *U, const float *Psi, int64_t ld,
                    const CdScratch &scr, int full) {
    if (nrect <= 0) return 0;
    constexpr int NB = snap_blocks_per_tile<T>();
    const int S = snapshot_parts(nrect, NB, q);
    SnapArgs<2, float> args{{SP, U}, {ld, ld}, {U, Psi}, {ld, ld}};
    snapshot<T, 2, float>(s, rects_dev, active, S, nrect, q, args, full, scr.partial);
    sum_snapshots<T>(s, active, nrect, S, scr.partial);
    return S;
}

void lambda_gauss_seidel(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                         int S, int64_t q, const double *Sigma, const double *Psi,
                         const double *GL, const double *Lam, double lamL, double *D,
                         double *dD, int *changed, const CdScratch &scr,
                         unsigned long long *counters, int esz) {
    if (nrect <= 0) return;
    lambda_gs_kernel<<<nrect, BLOCK, 0, s>>>(rects_dev, active, S, scr.partial, q, Sigma, Psi, GL,
                                             Lam, lamL, D, dD, changed, counters, esz);
    CGGM_LAUNCH_CHECK();
}

void lambda_update(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t q,
                   const double *Sigma, const double *dD, const int *changed, double *U) {
    if (nrect <= 0) return;
    const int64_t cols_per_wg = 64 * UPD_CHUNKS;
    dim3 grid((unsigned)((q + cols_per_wg - 1) / cols_per_wg), (unsigned)nrect, 2);
    lambda_u_update_kernel<double><<<grid, BLOCK, 0, s>>>(rects_dev, q, Sigma, dD, changed, U);
    CGGM_LAUNCH_CHECK();
}

void lambda_update(hipStream_t s, const TileRect *rects_dev, int nrect, int64_t ld,
                   const float *Sigma, const double *dD, const int *changed, float *U) {
    if (nrect <= 0) return;
    dim3 grid((unsigned)((ld + UPD32_COLS - 1) / UPD32_COLS), (unsigned)nrect, 2);
    lambda_u_update32_kernel<<<grid, BLOCK, 0, s>>>(rects_dev, ld, Sigma, dD, changed, U);
    CGGM_LAUNCH_CHECK();
}

void lambda_wave(hipStream_t s, const TileRect *rects_dev, const int *active, int nrect,
                 int64_t q, const double *Sigma, const double *Psi, const double *SP,
                 const double *GL, const double *Lam, double lamL, double *D, double *U,
                 double *dD, int *changed, const CdScratch &scr, const WaveProbe *probe,
                 const SweepF32 *f32) {
    if (nrect <= 0) return;
    const bool lo = f32 && f32->on;
    record(s, probe, 0);
    const int full = f32 ? f32->full_rects : -1;
    const int S = lo ? lambda_snapshot(s, rects_dev, active, nrect, q, f32->SP, f32->U,
                                       f32->Psi, f32->ldq, scr, full)
                     : lambda_snapshot(s, rects_dev, active, nrect, q, SP, U, Psi, scr, full);
    record(s, probe, 1);
    lambda_gauss_seidel(s, rects_dev, active, nrect, S, q, Sigma, Psi, GL, Lam, lamL, D, dD,
                        changed, scr, probe ? probe->counters : nullptr,
                        lo ? (int)sizeof(float) : (int)sizeof(double));
    record(s, probe, 2);
    if (lo)
        lambda_update(s, rects_dev, nrect, f32->ldq, f32->Sigma, dD, changed, f32->U);
    else
        lambda_update(s, rects_dev, nrect, q, Sigma, dD, changed, U);
    record(s, probe, 3);
}

}  // namespace cggm
