// engine.hip -- host engine and C ABI of the gfx950 alternating Newton
// coordinate descent solver (McCarter & Kim, AISTATS 2016, Algorithm 1).
//
// Control stays on the host; every arithmetic step runs in the kernels of
// la.hip, cd.hip and mixed.hip on the caller's stream.  The host reads back
// only scalars: the top-of-iteration statistics, the direction's decrease and
// the line-search quantities of each trial.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"
#include "schedule.hpp"
#include "solver.hpp"

// Workspace of cggm_objective_noalloc (file scope, one copy per device, held
// until the process ends).  Host code uses only its per-device address from
// hipGetSymbolAddress, never the name itself.
static __device__ __align__(256) char scratch[CGGM_NOALLOC_SCRATCH_BYTES];

namespace cggm {
namespace {

thread_local std::string g_last_error;

// ----------------------------------------------------------- kernels ---------
__global__ void fill_kernel(int64_t count, double v, double *x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) x[e] = v;
}

__global__ void widen_kernel(int64_t count, const float *a, double *b) {   // b = (double)a
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) b[e] = (double)a[e];
}

// Standard normal numbers from a counter (the tuner's synthetic inputs):
// SplitMix64 of (seed, index) gives two 53-bit uniforms, Box-Muller one
// normal.  Deterministic for a given seed.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void normal_kernel(int64_t count, uint64_t seed, double *x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const uint64_t a = splitmix64(seed ^ (2 * (uint64_t)e)), b = splitmix64(seed ^ (2 * (uint64_t)e + 1));
    const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740992.0);   // (0, 1]
    const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);           // [0, 1)
    x[e] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// V = Theta Sigma with Theta sparse (Sec. 3.2: V is kept from the rows of
// Sigma that Theta's nonzeros select).  One workgroup per (row i of Theta,
// block of VS_COLS columns): it scans Theta[i, :], stages the row's nonzeros
// (k, Theta_ik) in LDS in order, and accumulates Theta_ik Sigma[k, cols] in
// FP64 registers, k ascending (deterministic); the row is written once, in
// FP64 (V) or rounded to FP32 (V32, row length ld).  Rows of Sigma are read
// with consecutive lanes on consecutive columns.
constexpr int VS_PER_THREAD = 8;
constexpr int VS_COLS = BLOCK * VS_PER_THREAD;
constexpr int VS_CAP = 1024;

__global__ __launch_bounds__(BLOCK) void theta_sigma_sparse_kernel(
    int64_t q, int64_t ncb, const double *__restrict__ Theta, const double *__restrict__ Sigma,
    double *__restrict__ V, float *__restrict__ V32, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x / ncb;               // ncb column blocks per row
    const int64_t c0 = ((int64_t)blockIdx.x % ncb) * VS_COLS;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    __shared__ int kidx[VS_CAP];
    __shared__ double kval[VS_CAP];
    __shared__ int wsum[BLOCK / WAVE];
    double acc[VS_PER_THREAD];
#pragma unroll
    for (int u = 0; u < VS_PER_THREAD; ++u) acc[u] = 0.0;
    const double *row = Theta + i * q;
    int count = 0;                                  // staged nonzeros (uniform)
    auto flush = [&] {
        for (int j = 0; j < count; ++j) {
            const double tv = kval[j];
            const double *srow = Sigma + (int64_t)kidx[j] * q + c0 + tid;
#pragma unroll
            for (int u = 0; u < VS_PER_THREAD; ++u)
                if (c0 + tid + u * BLOCK < q) acc[u] = fma(tv, srow[u * BLOCK], acc[u]);
        }
        count = 0;
    };
    for (int64_t k0 = 0; k0 < q; k0 += BLOCK) {
        const int64_t k = k0 + tid;
        const double v = k < q ? row[k] : 0.0;
        const bool nz = v != 0.0;
        const uint64_t m = __ballot(nz);
        if (lane == 0) wsum[wid] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w2 = 0; w2 < BLOCK / WAVE; ++w2) {
            before += (w2 < wid) ? wsum[w2] : 0;
            total += wsum[w2];
        }
        if (count + total > VS_CAP) {                 // room for this block first
            flush();
            __syncthreads();                          // staged entries consumed
        }
        if (nz) {
            const int pos = count + before + __popcll(m & ((1ull << lane) - 1ull));
            kidx[pos] = (int)k;
            kval[pos] = v;
        }
        count += total;
        __syncthreads();                              // staged entries and wsum visible
    }
    flush();
#pragma unroll
    for (int u = 0; u < VS_PER_THREAD; ++u) {
        const int64_t col = c0 + tid + u * BLOCK;
        if (col < q) {
            if (V32)
                V32[i * ld + col] = (float)acc[u];
            else
                V[i * ld + col] = acc[u];
        }
    }
}

// y (rows x cols, ld ldy) = x (FP32, ld ldx) widened
__global__ void widen2d_kernel(int64_t rows, int64_t cols, const float *x, int64_t ldx,
                               double *y, int64_t ldy) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t r = e / cols, c = e % cols;
    y[r * ldy + c] = (double)x[r * ldx + c];
}

__global__ void add_kernel(int64_t count, const double *a, double *b) {   // b += a
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) b[e] += a[e];
}

// Nonzeros per row of a dense rows x cols matrix (one workgroup per row).
__global__ __launch_bounds__(BLOCK) void row_nnz_kernel(int64_t cols, const double *A,
                                                        int64_t *counts) {
    const int64_t r = blockIdx.x;
    int64_t c = 0;
    for (int64_t j = threadIdx.x; j < cols; j += BLOCK) c += (A[r * cols + j] != 0.0);
    __shared__ int64_t red[BLOCK];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[r] = red[0];
}

// CSR fill: one workgroup per row; chunks of BLOCK columns keep column order.
__global__ __launch_bounds__(BLOCK) void csr_fill_kernel(int64_t cols, const double *A,
                                                         const int64_t *rowptr, int32_t *col,
                                                         double *val) {
    const int64_t r = blockIdx.x;
    int64_t base = rowptr[r];
    __shared__ int scan[BLOCK];
    for (int64_t j0 = 0; j0 < cols; j0 += BLOCK) {
        const int64_t j = j0 + threadIdx.x;
        const double v = (j < cols) ? A[r * cols + j] : 0.0;
        const int nz = (j < cols && v != 0.0) ? 1 : 0;
        scan[threadIdx.x] = nz;
        __syncthreads();
        for (int s = 1; s < BLOCK; s <<= 1) {          // inclusive Hillis-Steele scan
            const int add = ((int)threadIdx.x >= s) ? scan[threadIdx.x - s] : 0;
            __syncthreads();
            scan[threadIdx.x] += add;
            __syncthreads();
        }
        if (nz) {
            const int64_t pos = base + scan[threadIdx.x] - 1;
            col[pos] = (int32_t)j;
            val[pos] = v;
        }
        const int total = scan[BLOCK - 1];
        __syncthreads();
        base += total;
    }
}

inline int nblk(int64_t count) { return (int)std::max<int64_t>(1, (count + BLOCK - 1) / BLOCK); }

void fill(hipStream_t s, int64_t count, double v, double *x) {
    fill_kernel<<<nblk(count), BLOCK, 0, s>>>(count, v, x);
    CGGM_LAUNCH_CHECK();
}

void check_dtype(int dtype) {
    if (dtype != CGGM_F64 && dtype != CGGM_F32) fail(CGGM_EINVAL, "dtype must be CGGM_F64 or CGGM_F32");
}

// X and Y as FP64 device arrays: the caller's when dtype is CGGM_F64, else
// the exact FP64 widening of the caller's FP32 arrays into X64 / Y64.
std::pair<const double *, const double *> fp64_inputs(hipStream_t s, int dtype, int64_t n,
                                                      int64_t p, int64_t q, const void *X,
                                                      const void *Y, double *X64, double *Y64) {
    if (dtype == CGGM_F64) return {(const double *)X, (const double *)Y};
    widen_kernel<<<nblk(n * p), BLOCK, 0, s>>>(n * p, (const float *)X, X64);
    CGGM_LAUNCH_CHECK();
    widen_kernel<<<nblk(n * q), BLOCK, 0, s>>>(n * q, (const float *)Y, Y64);
    CGGM_LAUNCH_CHECK();
    return {X64, Y64};
}

// ----------------------------------------------------------- device arena ----
struct Arena {
    char *base = nullptr;
    size_t used = 0, cap = 0;
    bool measure = false;
    template <class Tp>
    Tp *take(int64_t count) {
        const size_t bytes = ((size_t)std::max<int64_t>(count, 1) * sizeof(Tp) + 255) & ~size_t(255);
        Tp *p = measure ? nullptr : reinterpret_cast<Tp *>(base + used);
        used += bytes;
        return p;
    }
};

struct DeviceBuffer {
    void *p = nullptr;
    ~DeviceBuffer() {
        if (p) (void)hipFree(p);
    }
};

// --------------------------------------------------------------- workspace ---
struct Work {
    int64_t n = 0, p = 0, q = 0;
    double *Sxx, *Sxy, *Syy;                       // statistics
    double *Lam, *LamT, *L, *Lt, *Sig, *Psi, *SP, *GL, *D, *U;   // q x q
    double *Wd, *Wdt;                              // diagonal-block inverses of L, Lt
    double *Th, *ThOld, *GT, *V;                   // p x q
    double *A, *R, *At, *Zt;                       // n x q, q x n
    double *dT, *dD;                               // per-wave tile deltas
    double *partials, *scal;                       // reduction scratch, device scalars
    int *flag, *changed;
    unsigned long long *kctr;                      // sweep counters [2][8]
    CdScratch cd;                                  // split-snapshot scratch
    int *act_theta, *act_lambda;                   // per-rect activity of a sweep
    TileRect *rects_theta, *rects_lambda;
    int max_tiles = 0;
    __bf16 *split_Th = nullptr, *split_Sig = nullptr;   // mixed mode: BF16 pieces
    // mixed mode: FP32 copies of the operands the CD sweeps stream
    float *SP32 = nullptr, *Psi32 = nullptr, *Sig32 = nullptr, *U32 = nullptr;
    float *Sxx32 = nullptr, *V32 = nullptr;
    double *X64 = nullptr, *Y64 = nullptr;          // FP64 copies of FP32 inputs
    int64_t sxx_ld = 0;     // row length of Sxx as the Theta sweep reads it
    float *Sxx32slab = nullptr;                     // block-wise mode, mixed: FP32 slab
};

constexpr int NSCAL = 64;

// Layout of the workspace; with a.measure it only sizes it.
// slab_cols == 0: the full Sxx (p x p); otherwise the block-wise mode's slab
// of slab_cols columns of Sxx (p x slab_cols) in its place.
void layout(Arena &a, Work &w, int64_t n, int64_t p, int64_t q, int64_t ntheta_rects,
            int64_t nlambda_rects, int max_tiles, bool mixed = false, bool f32 = false,
            bool f32_inputs = false, int64_t slab_cols = 0) {
    const int64_t qq = q * q, pq = p * q, nq = n * q;
    w.n = n, w.p = p, w.q = q;
    w.sxx_ld = slab_cols ? slab_cols : p;
    w.Sxx = a.take<double>(p * w.sxx_ld);
    w.Sxy = a.take<double>(pq);
    w.Syy = a.take<double>(qq);
    w.Lam = a.take<double>(qq);
    w.LamT = a.take<double>(qq);
    w.L = a.take<double>(qq);
    w.Lt = a.take<double>(qq);
    w.Sig = a.take<double>(qq);
    w.Psi = a.take<double>(qq);
    w.SP = a.take<double>(qq);
    w.GL = a.take<double>(qq);
    w.D = a.take<double>(qq);
    w.U = a.take<double>(qq);
    w.Wd = a.take<double>(diag_inv_count(q));
    w.Wdt = a.take<double>(diag_inv_count(q));
    w.Th = a.take<double>(pq);
    w.ThOld = a.take<double>(pq);
    w.GT = a.take<double>(pq);
    w.V = a.take<double>(pq);
    w.A = a.take<double>(nq);
    w.R = a.take<double>(nq);
    w.At = a.take<double>(nq);
    w.Zt = a.take<double>(nq);
    w.max_tiles = max_tiles;
    w.dT = a.take<double>((int64_t)max_tiles * THETA_TILE * THETA_TILE);
    w.dD = a.take<double>((int64_t)max_tiles * LAMBDA_TILE * LAMBDA_TILE);
    w.partials = a.take<double>(REDUCE_BLOCKS * 8);
    w.scal = a.take<double>(NSCAL);
    w.flag = a.take<int>(4);
    w.changed = a.take<int>(max_tiles);
    w.kctr = a.take<unsigned long long>(16);
    w.cd.partial = a.take<double>((int64_t)max_tiles * CD_MAX_PARTS * THETA_TILE * THETA_TILE);
    w.act_theta = a.take<int>(ntheta_rects);
    w.act_lambda = a.take<int>(nlambda_rects);
    w.rects_theta = a.take<TileRect>(ntheta_rects);
    w.rects_lambda = a.take<TileRect>(nlambda_rects);
    if (mixed) {
        w.split_Th = a.take<__bf16>(3 * p * split3_stride(q));
        w.split_Sig = a.take<__bf16>(3 * q * split3_stride(q));
    }
    if (f32) {
        const int64_t lq = f32_ld(q), lp = f32_ld(p);
        w.SP32 = a.take<float>(q * lq);
        w.Psi32 = a.take<float>(q * lq);
        w.Sig32 = a.take<float>(q * lq);
        w.U32 = a.take<float>(q * lq);
        if (slab_cols)
            w.Sxx32slab = a.take<float>(p * slab_cols);
        else
            w.Sxx32 = a.take<float>(p * lp);
        w.V32 = a.take<float>(p * lq);
    }
    if (f32_inputs) {
        w.X64 = a.take<double>(n * p);
        w.Y64 = a.take<double>(n * q);
    }
}

// Scalars read back at the top of an iteration (offsets into Work::scal).
enum {
    S_LAM = 0,       // 5: tr(Syy Lam), |Lam|_1, subgrad, m, nnz
    S_THETA = 5,     // 5: <Sxy, Theta>, |Theta|_1, subgrad, m, nnz
    S_AR = 10,       // <A, R>
    S_LOGDET = 11,   // 2: logdet, bad
    S_DIR = 13,      // 2: <G, D>, sum |Lam + D| - |Lam|
    S_TRIAL = 15,    // 2: tr(Syy T), |T|_1
    S_TLOGDET = 17,  // 2
    S_ZZ = 19,       // |L^{-1} A^T|_F^2
    S_NONFIN = 20,   // 2: non-finite counts of X and Y
};

// Captured launch sequences of the tiled sweeps (options.graphs): the wave
// loop of a sweep -- a fixed sequence of kernel launches for a given schedule
// -- is recorded once into a HIP graph and replayed on later sweeps, which
// saves the host-side cost of hundreds of small launches per pass.  Every
// kernel argument that can differ between sweeps is part of the key: the
// schedule, the buffer the swapped parameter currently lives in (the line
// search swaps Lambda with its trial), the penalty and the precision of the
// operands.  At most MAX graphs are kept (the oldest is dropped).
struct SweepGraphs {
    static constexpr size_t MAX = 32;
    struct Entry {
        const Schedule *sch;
        const void *buf;
        double lam;
        bool f32;
        hipGraphExec_t exec;
    };
    std::vector<Entry> cache;
    int64_t captured = 0, replayed = 0;
    // The launches are recorded on a stream of the library's own (a caller's
    // stream may be the legacy default stream, which cannot be captured);
    // recording executes nothing, and the graph is then launched on the
    // caller's stream.
    hipStream_t cap = nullptr;
    ~SweepGraphs() {
        for (auto &e : cache)
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
    // launch(stream) issues the wave loop's kernels on `stream`.
    template <class F>
    void run(hipStream_t s, const Schedule *sch, const void *buf, double lam, bool f32,
             F &&launch) {
        for (auto &e : cache)
            if (e.sch == sch && e.buf == buf && e.lam == lam && e.f32 == f32) {
                CGGM_HIP(hipGraphLaunch(e.exec, s));
                ++replayed;
                return;
            }
        if (!cap) CGGM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        CGGM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
            launch(cap);
        } catch (...) {
            if (hipStreamEndCapture(cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            throw;
        }
        CGGM_HIP(hipStreamEndCapture(cap, &g));
        hipGraphExec_t exec = nullptr;
        const hipError_t err = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        CGGM_HIP(err);
        if (cache.size() >= MAX) {
            (void)hipGraphExecDestroy(cache.front().exec);
            cache.erase(cache.begin());
        }
        cache.push_back({sch, buf, lam, f32, exec});
        ++captured;
        CGGM_HIP(hipGraphLaunch(exec, s));
    }
};

struct Ctx {
    hipStream_t s;
    Work &w;
    double lamL, lamT;
    bool mixed = false;   // split-BF16 V and FP32 sweep operands
    SweepGraphs *graphs = nullptr;   // capture and replay the sweeps' wave loops
    double theta_density = -1.0;     // nnz(Theta) / (p q) of the iterate (< 0: unknown)
    bool f32() const { return mixed && w.Sig32 != nullptr; }
};

// V = Theta Sigma: FP64 MFMA, or in mixed mode from the BF16 pieces of Theta
// and Sigma (Sigma symmetric: its rows are the columns the product needs) into
// the FP32 V the mixed Theta sweep maintains.
// Fraction of nonzeros in Theta below which V = Theta Sigma is formed as a
// sparse-by-dense product (about 16 nnz q bytes of Sigma rows and Theta scans
// against 2 p q^2 flops of the dense product).
constexpr double SPARSE_V_DENSITY = 0.02;

void theta_sigma(Ctx &c) {
    Work &w = c.w;
    if (c.theta_density >= 0.0 && c.theta_density < SPARSE_V_DENSITY) {
        const int64_t ncb = (w.q + VS_COLS - 1) / VS_COLS;
        const bool to32 = c.f32();
        theta_sigma_sparse_kernel<<<(unsigned)(w.p * ncb), BLOCK, 0, c.s>>>(
            w.q, ncb, w.Th, w.Sig, to32 ? nullptr : w.V, to32 ? w.V32 : nullptr,
            to32 ? f32_ld(w.q) : w.q);
        CGGM_LAUNCH_CHECK();
        return;
    }
    if (!c.mixed) {
        gemm(c.s, false, false, w.p, w.q, w.q, 1.0, w.Th, w.q, w.Sig, w.q, 0.0, w.V, w.q);
        return;
    }
    split3(c.s, w.p, w.q, w.Th, w.q, w.split_Th);
    split3(c.s, w.q, w.q, w.Sig, w.q, w.split_Sig);
    if (c.f32())
        gemm_split3_nt(c.s, w.p, w.q, w.q, w.split_Th, w.split_Sig, w.V32, f32_ld(w.q));
    else
        gemm_split3_nt(c.s, w.p, w.q, w.q, w.split_Th, w.split_Sig, w.V, w.q);
}

// Operands of a sweep in the current precision.
SweepF32 sweep_operands(const Ctx &c) {
    SweepF32 f;
    if (!c.f32()) return f;
    const Work &w = c.w;
    f.on = true;
    f.ldq = f32_ld(w.q);
    f.ldx = f32_ld(w.p);
    f.SP = w.SP32;
    f.Psi = w.Psi32;
    f.Sigma = w.Sig32;
    f.Sxx = w.Sxx32;
    f.U = w.U32;
    f.V = w.V32;
    return f;
}

// Sigma of the current factor; in mixed mode also its FP32 copy.
void refresh_sigma(Ctx &c) {
    Work &w = c.w;
    spd_inverse_from_cholesky(c.s, w.q, w.L, w.Wd, w.U, w.Sig);
    if (c.f32()) to_f32(c.s, w.q, w.q, w.Sig, w.q, w.Sig32, f32_ld(w.q));
}

// Rounding allowance of an FP64 objective evaluation in the Armijo test and
// the Theta descent guard.
constexpr double F_ROUNDING = 1e-14;

// Sxx = X^T X / n, Sxy = X^T Y / n, Syy = Y^T Y / n (uncentred, Sec. 2.1).
// In the block-wise mode Sxx is not formed here: the Theta sweep forms the
// columns of a row group at a time (Sec. 4.2).
void statistics(Ctx &c, const double *X, const double *Y, bool full_sxx = true) {
    Work &w = c.w;
    const double inv_n = 1.0 / (double)w.n;
    if (full_sxx) {
        gemm(c.s, true, false, w.p, w.p, w.n, inv_n, X, w.p, X, w.p, 0.0, w.Sxx, w.p,
             UPLO_LOWER);
        symmetrize_from_lower(c.s, w.p, w.Sxx);
    }
    gemm(c.s, true, false, w.p, w.q, w.n, inv_n, X, w.p, Y, w.q, 0.0, w.Sxy, w.q);
    gemm(c.s, true, false, w.q, w.q, w.n, inv_n, Y, w.q, Y, w.q, 0.0, w.Syy, w.q, UPLO_LOWER);
    symmetrize_from_lower(c.s, w.q, w.Syy);
}

// A = X Theta, R = A Sigma; reductions <A, R>, <Sxy, Theta>-block stats use them.
void theta_products(Ctx &c, const double *X) {
    Work &w = c.w;
    gemm(c.s, false, false, w.n, w.q, w.p, 1.0, X, w.p, w.Th, w.q, 0.0, w.A, w.q);
    gemm(c.s, false, false, w.n, w.q, w.q, 1.0, w.A, w.q, w.Sig, w.q, 0.0, w.R, w.q);
}

// Psi = R^T R / n, G_Lambda = Syy - Sigma - Psi, SP = Sigma + Psi,
// G_Theta = 2 Sxy + (2/n) X^T R  (= 2 Sxy + 2 Sxx Theta Sigma), Eq. (3).
void gradients(Ctx &c, const double *X) {
    Work &w = c.w;
    const double inv_n = 1.0 / (double)w.n;
    gemm(c.s, true, false, w.q, w.q, w.n, inv_n, w.R, w.q, w.R, w.q, 0.0, w.Psi, w.q,
         UPLO_LOWER);
    symmetrize_from_lower(c.s, w.q, w.Psi);
    assemble_lambda_gradient(c.s, w.q, w.Syy, w.Sig, w.Psi, w.GL, w.SP);
    scale_copy(c.s, w.p * w.q, 2.0, w.Sxy, w.GT);
    gemm(c.s, true, false, w.p, w.q, w.n, 2.0 * inv_n, X, w.p, w.R, w.q, 1.0, w.GT, w.q);
    if (c.f32()) {
        to_f32(c.s, w.q, w.q, w.SP, w.q, w.SP32, f32_ld(w.q));
        to_f32(c.s, w.q, w.q, w.Psi, w.q, w.Psi32, f32_ld(w.q));
    }
}

struct TopStats {
    double f, subgrad, l1, trS, sxyT, l1L, l1T, ar, logdet;
    int64_t mL, mT, nnzL, nnzT;
};

// Objective and the Theta-side scalars after A, R are current (Lambda side
// taken from stats already on the device).
TopStats read_top(Ctx &c, bool with_gradient_stats) {
    Work &w = c.w;
    double h[NSCAL];
    CGGM_HIP(hipMemcpyAsync(h, w.scal, sizeof(h), hipMemcpyDeviceToHost, c.s));
    CGGM_HIP(hipStreamSynchronize(c.s));
    TopStats t{};
    t.trS = h[S_LAM + 0];
    t.l1L = h[S_LAM + 1];
    t.sxyT = h[S_THETA + 0];
    t.l1T = h[S_THETA + 1];
    t.ar = h[S_AR];
    t.logdet = h[S_LOGDET];
    t.f = -t.logdet + t.trS + 2.0 * t.sxyT + t.ar / (double)w.n + c.lamL * t.l1L +
          c.lamT * t.l1T;
    if (with_gradient_stats) {
        t.subgrad = h[S_LAM + 2] + h[S_THETA + 2];
        t.mL = (int64_t)h[S_LAM + 3];
        t.mT = (int64_t)h[S_THETA + 3];
        t.nnzL = (int64_t)h[S_LAM + 4];
        t.nnzT = (int64_t)h[S_THETA + 4];
    }
    t.l1 = t.l1L + t.l1T;
    return t;
}

// Optional per-stage kernel timing of the CD sweeps: intervals between pairs
// of events recorded on the stream a stage runs on, summed per stage
// (0 snapshot, 1 Gauss-Seidel, 2 update) when the events are done.
struct KernelTimer {
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Interval {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Interval> pending;
    unsigned long long *counters = nullptr;
    int64_t waves = 0, pending_waves = 0;
    double ms[3] = {0.0, 0.0, 0.0};
    bool enabled = false;
    void init(unsigned long long *ctr) {
        counters = ctr;
        enabled = true;
    }
    ~KernelTimer() {
        for (auto &e : pool)
            if (e) (void)hipEventDestroy(e);
    }
    bool on() const { return enabled; }
    hipEvent_t event() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            CGGM_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    void interval(int stage, hipEvent_t a, hipEvent_t b) { pending.push_back({stage, a, b}); }
    // Events of one single-stream wave: snapshot [0,1), Gauss-Seidel [1,2), update [2,3).
    WaveProbe probe() {
        WaveProbe p;
        for (int j = 0; j < 4; ++j) p.ev[j] = event();
        for (int j = 0; j < 3; ++j) interval(j, p.ev[j], p.ev[j + 1]);
        p.counters = counters;
        ++pending_waves;
        return p;
    }
    // Sum the pending intervals (their events must be done) and recycle the events.
    void collect() {
        for (const Interval &iv : pending) {
            float m = 0.f;
            CGGM_HIP(hipEventElapsedTime(&m, iv.a, iv.b));
            ms[iv.stage] += m;
        }
        pending.clear();
        used = 0;
        waves += pending_waves;
        pending_waves = 0;
    }
};

// Block-wise mode (Sec. 4.2, Algorithm 2): the Theta sweep holds the Sxx
// columns of one group of `rows` consecutive rows (a slab, p x rows, formed
// from X on the matrix cores as X^T X[:, group] / n when a wave of that group
// needs it; Sxx is symmetric, so these are also the rows a tile of the group
// reads) instead of the whole p x p matrix.  The waves of a group are
// consecutive, so each group's slab is formed at most once per pass, and
// groups without an active coordinate are skipped altogether (neither their
// slab nor their waves run).
struct SxxSlab {
    bool on = false;
    int64_t rows = 0;          // Sxx columns per group (a multiple of the tile edge)
    const double *X = nullptr;
    int64_t cur = -1;          // group whose columns the slab holds
    std::vector<int> act;      // host copy of the rect activity of the sweep
    int64_t formed = 0;        // slabs formed (statistics)
};

void form_slab(Ctx &c, SxxSlab &sl, int64_t g) {
    Work &w = c.w;
    const int64_t r0 = g * sl.rows, cols = std::min(w.p, r0 + sl.rows) - r0;
    gemm(c.s, true, false, w.p, cols, w.n, 1.0 / (double)w.n, sl.X, w.p, sl.X + r0, w.p, 0.0,
         w.Sxx, w.sxx_ld);
    if (w.Sxx32slab)
        to_f32(c.s, w.p, cols, w.Sxx, w.sxx_ld, w.Sxx32slab, w.sxx_ld);
    sl.cur = g;
    ++sl.formed;
}

// The 64 x 64 rects of the wave [b, e) of `sch`.  The snapshot reads operands
// through buffer resources when there is one: the schedule then has 64-edge
// tiles, and every smaller one ends at the matrix edge.
int full_rects(const Schedule &sch, int b, int e) {
    int n = 0;
    for (int r = b; r < e; ++r) {
        const TileRect &t = sch.rects[r];
        n += (t.r1 - t.r0 == THETA_TILE && t.c1 - t.c0 == THETA_TILE) ? 1 : 0;
    }
    return n;
}

// One CD pass over S_Theta; the activity of the tiles is taken on the first
// pass (pass == 0) from the top-of-iteration gradient, further passes reuse it.
void run_theta_sweep(Ctx &c, const Schedule &sch, KernelTimer *kt = nullptr, int pass = 0,
                     SxxSlab *sl = nullptr) {
    Work &w = c.w;
    SweepF32 f32 = sweep_operands(c);
    if (pass == 0)
        theta_activity(c.s, w.rects_theta, (int)sch.rects.size(), w.q, w.GT, w.Th, c.lamT,
                       w.act_theta);
    const bool block = sl && sl->on;
    if (block && pass == 0) {
        sl->act.resize(sch.rects.size());
        CGGM_HIP(hipMemcpyAsync(sl->act.data(), w.act_theta, sizeof(int) * sch.rects.size(),
                                hipMemcpyDeviceToHost, c.s));
        CGGM_HIP(hipStreamSynchronize(c.s));
    }
    if (c.graphs && !block && !(kt && kt->on())) {
        c.graphs->run(c.s, &sch, w.Th, c.lamT, f32.on, [&](hipStream_t st) {
            for (int k = 0; k < sch.waves(); ++k) {
                const int b = sch.wave_start[k], e = sch.wave_start[k + 1];
                f32.full_rects = full_rects(sch, b, e);
                theta_wave(st, w.rects_theta + b, w.act_theta + b, e - b, w.p, w.q, w.Sxx, w.p,
                           w.Sxy, w.Sig, w.V, w.GT, w.Th, c.lamT, w.dT, w.changed, w.cd, nullptr,
                           &f32);
            }
        });
        return;
    }
    for (int k = 0; k < sch.waves(); ++k) {
        const int b = sch.wave_start[k], e = sch.wave_start[k + 1];
        const double *Sxx = w.Sxx;
        int64_t ldx = w.p;
        if (block) {
            bool any = false;
            for (int r = b; r < e && !any; ++r) any = sl->act[r] != 0;
            if (!any) continue;
            const int64_t g = sch.rects[b].r0 / sl->rows;
            if (g != sl->cur) form_slab(c, *sl, g);
            // column i of the group at Sxx[k * ldx + i]: the slab shifted by the
            // group's first column
            Sxx = w.Sxx - g * sl->rows;
            ldx = w.sxx_ld;
            if (f32.on) {
                f32.Sxx = w.Sxx32slab - g * sl->rows;
                f32.ldx = w.sxx_ld;
            }
        }
        WaveProbe pr;
        if (kt && kt->on()) pr = kt->probe();
        f32.full_rects = full_rects(sch, b, e);
        theta_wave(c.s, w.rects_theta + b, w.act_theta + b, e - b, w.p, w.q, Sxx, ldx, w.Sxy,
                   w.Sig, w.V, w.GT, w.Th, c.lamT, w.dT, w.changed, w.cd,
                   (kt && kt->on()) ? &pr : nullptr, &f32);
    }
}

// One CD pass over S_Lambda for the Newton direction; D and U start at zero
// on the first pass and carry over to further passes (pass > 0).
void run_lambda_sweep(Ctx &c, const Schedule &sch, KernelTimer *kt = nullptr, int pass = 0) {
    Work &w = c.w;
    SweepF32 f32 = sweep_operands(c);
    if (pass == 0) {
        fill(c.s, w.q * w.q, 0.0, w.D);
        if (f32.on)
            fill_f32(c.s, w.q * f32_ld(w.q), 0.0f, w.U32);
        else
            fill(c.s, w.q * w.q, 0.0, w.U);
        lambda_activity(c.s, w.rects_lambda, (int)sch.rects.size(), w.q, w.GL, w.Lam, c.lamL,
                        w.act_lambda);
    }
    if (c.graphs && !(kt && kt->on())) {
        c.graphs->run(c.s, &sch, w.Lam, c.lamL, f32.on, [&](hipStream_t st) {
            for (int k = 0; k < sch.waves(); ++k) {
                const int b = sch.wave_start[k], e = sch.wave_start[k + 1];
                f32.full_rects = full_rects(sch, b, e);
                lambda_wave(st, w.rects_lambda + b, w.act_lambda + b, e - b, w.q, w.Sig, w.Psi,
                            w.SP, w.GL, w.Lam, c.lamL, w.D, w.U, w.dD, w.changed, w.cd, nullptr,
                            &f32);
            }
        });
        return;
    }
    for (int k = 0; k < sch.waves(); ++k) {
        const int b = sch.wave_start[k], e = sch.wave_start[k + 1];
        WaveProbe pr;
        if (kt && kt->on()) pr = kt->probe();
        f32.full_rects = full_rects(sch, b, e);
        lambda_wave(c.s, w.rects_lambda + b, w.act_lambda + b, e - b, w.q, w.Sig, w.Psi, w.SP,
                    w.GL, w.Lam, c.lamL, w.D, w.U, w.dD, w.changed, w.cd,
                    (kt && kt->on()) ? &pr : nullptr, &f32);
    }
}

struct ResultImpl {
    int64_t p = 0, q = 0, nnzL = 0, nnzT = 0;
    int iters = 0, status = 0;
    double f = 0.0;
    double *Lam = nullptr, *Th = nullptr;          // dense, device
    int64_t *L_rowptr = nullptr, *T_rowptr = nullptr;
    int32_t *L_col = nullptr, *T_col = nullptr;
    double *L_val = nullptr, *T_val = nullptr;
    ~ResultImpl() {
        for (void *ptr : {(void *)Lam, (void *)Th, (void *)L_rowptr, (void *)T_rowptr,
                          (void *)L_col, (void *)T_col, (void *)L_val, (void *)T_val})
            if (ptr) (void)hipFree(ptr);
    }
};

void to_csr(hipStream_t s, int64_t rows, int64_t cols, const double *A, int64_t **rowptr,
            int32_t **col, double **val, int64_t *nnz) {
    CGGM_HIP(hipMalloc(rowptr, sizeof(int64_t) * (rows + 1)));
    std::vector<int64_t> counts(rows), ptr(rows + 1, 0);
    row_nnz_kernel<<<(unsigned)rows, BLOCK, 0, s>>>(cols, A, *rowptr);
    CGGM_LAUNCH_CHECK();
    CGGM_HIP(hipMemcpyAsync(counts.data(), *rowptr, sizeof(int64_t) * rows, hipMemcpyDeviceToHost,
                            s));
    CGGM_HIP(hipStreamSynchronize(s));
    for (int64_t r = 0; r < rows; ++r) ptr[r + 1] = ptr[r] + counts[r];
    *nnz = ptr[rows];
    CGGM_HIP(hipMemcpyAsync(*rowptr, ptr.data(), sizeof(int64_t) * (rows + 1),
                            hipMemcpyHostToDevice, s));
    CGGM_HIP(hipMalloc(col, sizeof(int32_t) * std::max<int64_t>(*nnz, 1)));
    CGGM_HIP(hipMalloc(val, sizeof(double) * std::max<int64_t>(*nnz, 1)));
    csr_fill_kernel<<<(unsigned)rows, BLOCK, 0, s>>>(cols, A, *rowptr, *col, *val);
    CGGM_LAUNCH_CHECK();
    CGGM_HIP(hipStreamSynchronize(s));
}

void check_sizes(int64_t n, int64_t p, int64_t q) {
    if (n < 1 || p < 1 || q < 1) fail(CGGM_EINVAL, "n, p and q must be >= 1");
    if (p > INT32_MAX || q > INT32_MAX) fail(CGGM_EINVAL, "p and q must fit in int32");
}

void check_lambda(double lamL, double lamT) {
    if (!(lamL >= 0.0) || !(lamT >= 0.0) || !isfinite(lamL) || !isfinite(lamT))
        fail(CGGM_EINVAL, "penalties must be finite and >= 0");
}

// Non-finite entries of X and Y -> CGGM_EINVAL.
void check_finite(Ctx &c, const double *X, const double *Y) {
    Work &w = c.w;
    reduce_nonfinite(c.s, w.n * w.p, X, w.partials, w.scal + S_NONFIN);
    reduce_nonfinite(c.s, w.n * w.q, Y, w.partials, w.scal + S_NONFIN + 1);
    double h[2];
    CGGM_HIP(hipMemcpyAsync(h, w.scal + S_NONFIN, sizeof(h), hipMemcpyDeviceToHost, c.s));
    CGGM_HIP(hipStreamSynchronize(c.s));
    if (h[0] != 0.0 || h[1] != 0.0) fail(CGGM_EINVAL, "X or Y has non-finite entries");
}

// Tile edges of the Lambda and Theta sweeps; `tile` > 0 caps both.
std::pair<int, int> tile_edges(int tile) {
    if (tile <= 0) return {LAMBDA_TILE, THETA_TILE};
    if (tile > THETA_TILE) fail(CGGM_EINVAL, "tile must be <= 64");
    return {std::min(tile, LAMBDA_TILE), std::min(tile, THETA_TILE)};
}

// ------------------------------------------------------------------ solve ----
cggm_options checked_options(const cggm_options *opt_in) {
    cggm_options opt;
    cggm_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.max_iter < 0 || opt.max_ls < 1 || !(opt.ls_beta > 0.0 && opt.ls_beta < 1.0) ||
        !(opt.ls_sigma > 0.0 && opt.ls_sigma < 1.0) || opt.stall_iters < 0 ||
        opt.lambda_passes < 0 || opt.mixed_min_q < 0 || opt.theta_passes < 1 ||
        opt.split_level < 0 || opt.split_level > 6 || (opt.blockwise != 0 && opt.blockwise != 1) ||
        (opt.graphs != 0 && opt.graphs != 1) ||
        (opt.precision != CGGM_PRECISION_FP64 && opt.precision != CGGM_PRECISION_MIXED) ||
        (opt.sweep != CGGM_SWEEP_TILED && opt.sweep != CGGM_SWEEP_SEQUENTIAL))
        fail(CGGM_EINVAL, "invalid options");
    return opt;
}

}  // namespace

struct Solver::Impl {
    int64_t n, p, q;
    int dtype;
    cggm_options opt;
    bool mixed, seq;
    hipStream_t s;
    Schedule th_sched, la_sched, th_safe, la_safe;   // *_safe: one tile per wave
    // th_sched / la_sched with every wave split into 2^level sub-waves
    // (level 1 .. MAX_SPLIT_LEVEL), built on first use.
    static constexpr int MAX_SPLIT_LEVEL = 6;
    std::vector<std::unique_ptr<Schedule>> th_split, la_split;
    int max_tiles = 1;
    size_t bytes = 0;
    DeviceBuffer own;
    Work w;
    const double *X = nullptr;
    KernelTimer kt_lambda, kt_theta;
    SxxSlab slab;                 // block-wise mode: the Theta sweep's Sxx columns
    SweepGraphs graphs;           // options.graphs: captured sweep launch sequences
    hipEvent_t ev[5] = {};
    std::chrono::steady_clock::time_point t0;
    int trace_len = 0;
    bool loaded = false, started = false;

    Impl(int64_t n_, int64_t p_, int64_t q_, const cggm_options *o, hipStream_t st, int dt)
        : n(n_), p(p_), q(q_), dtype(dt), opt(checked_options(o)), s(st) {
        check_sizes(n, p, q);
        check_dtype(dtype);
        // Passes of the Lambda direction, chosen by the conditioning of its
        // subproblem: with fewer samples than a quarter of the outputs, Syy
        // has low rank and the coordinate descent needs more passes for a
        // useful Newton direction (measured on the chain generator: 4 passes
        // best at q = 2000, n = 500; 6 passes best at q = 4000, n = 200, where
        // they reach a 1e-6 gap in 97 s against > 200 s with 4).
        if (opt.lambda_passes == 0) opt.lambda_passes = (4 * n >= q) ? 4 : 6;
        mixed = opt.precision == CGGM_PRECISION_MIXED && q >= opt.mixed_min_q;
        seq = opt.sweep == CGGM_SWEEP_SEQUENTIAL;
        const auto [tileL, tileT] = tile_edges(opt.tile);
        if (opt.blockwise) {
            // Sxx columns per group from the budget (Sec. 4.2: as many columns as
            // fit), whole row tiles, at least one: 8 bytes per entry, 12 in the
            // mixed mode (FP32 copy).
            const size_t budget = opt.sxx_cache_bytes ? opt.sxx_cache_bytes : (size_t(2) << 30);
            const int64_t per_tile = (int64_t)tileT * p * (mixed ? 12 : 8);
            const int64_t P = (p + tileT - 1) / tileT;
            const int64_t G = std::max<int64_t>(1, std::min<int64_t>(P, (int64_t)budget / per_tile));
            slab.on = true;
            slab.rows = G * tileT;
            th_sched = seq ? theta_schedule(p, q, tileT, true)
                           : theta_schedule_grouped(p, q, tileT, G);
        } else {
            th_sched = theta_schedule(p, q, tileT, seq);
        }
        la_sched = lambda_schedule(q, tileL, seq);
        for (auto [src, dst] : {std::pair<Schedule *, Schedule *>{&th_sched, &th_safe},
                                std::pair<Schedule *, Schedule *>{&la_sched, &la_safe}}) {
            dst->wave_start.push_back(0);
            for (const TileRect &r : src->rects) {
                dst->rects.push_back(r);
                dst->finish_wave();
            }
        }
        max_tiles = std::max(1, std::max(th_sched.max_wave, la_sched.max_wave));
        Arena sizer;
        sizer.measure = true;
        lay(sizer);
        bytes = sizer.used;
    }
    ~Impl() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void lay(Arena &a) {
        layout(a, w, n, p, q, (int64_t)th_sched.rects.size(), (int64_t)la_sched.rects.size(),
               max_tiles, mixed, mixed, dtype == CGGM_F32,
               slab.on ? std::min(slab.rows, (p + 63) / 64 * 64) : 0);
    }
    const Schedule &split_sched(std::vector<std::unique_ptr<Schedule>> &cache,
                                const Schedule &base, int level) {
        if (level == 0 || seq) return base;
        if ((int)cache.size() <= level) cache.resize(level + 1);
        if (!cache[level]) cache[level] = std::make_unique<Schedule>(split_waves(base, 1 << level));
        return *cache[level];
    }
    double ms_since(std::chrono::steady_clock::time_point a) const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a)
            .count();
    }
    void bind(void *base) {
        if (!base) fail(CGGM_EINVAL, "NULL workspace");
        Arena arena;
        arena.base = (char *)base;
        lay(arena);
        CGGM_HIP(hipMemcpyAsync(w.rects_theta, th_sched.rects.data(),
                                sizeof(TileRect) * th_sched.rects.size(), hipMemcpyHostToDevice,
                                s));
        CGGM_HIP(hipMemcpyAsync(w.rects_lambda, la_sched.rects.data(),
                                sizeof(TileRect) * la_sched.rects.size(), hipMemcpyHostToDevice,
                                s));
        // The host vectors are read by the copies above; they live as long as
        // the solver, and load() synchronises the stream before returning.
        for (auto &e : ev) CGGM_HIP(hipEventCreate(&e));
    }
    void allocate() {
        if (opt.workspace_budget && bytes > opt.workspace_budget)
            fail(CGGM_ENOMEM, "workspace of " + std::to_string(bytes) +
                                  " bytes exceeds the budget of " +
                                  std::to_string(opt.workspace_budget));
        if (hipMalloc(&own.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            own.p = nullptr;
            fail(CGGM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        bind(own.p);
    }
    void load(const void *X_in, const void *Y_in) {
        if (!X_in || !Y_in) fail(CGGM_EINVAL, "NULL pointer argument");
        const auto [X_, Y] = fp64_inputs(s, dtype, n, p, q, X_in, Y_in, w.X64, w.Y64);
        X = X_;
        Ctx c{s, w, 0.0, 0.0, mixed};
        check_finite(c, X, Y);                 // synchronises the stream
        if (opt.kstats) {
            fill(s, 16, 0.0, reinterpret_cast<double *>(w.kctr));   // all-zero bits
            kt_lambda.init(w.kctr);
            kt_theta.init(w.kctr + 8);
        }
        t0 = std::chrono::steady_clock::now();
        statistics(c, X, Y, !slab.on);
        slab.X = X;
        slab.cur = -1;
        if (c.f32()) {
            if (!slab.on) to_f32(s, p, p, w.Sxx, p, w.Sxx32, f32_ld(p));
            fill_f32(s, p * f32_ld(q), 0.0f, w.V32);   // the padding columns stay zero
        }
        loaded = true;
    }
    void start() {
        if (!loaded) fail(CGGM_EINVAL, "start before load");
        const int64_t qq = q * q, pq = p * q;
        Ctx c{s, w, 0.0, 0.0, mixed};
        // Algorithm 1: Theta = 0, Lambda = I (or the warm start).
        if (opt.warm_Lambda) {
            CGGM_HIP(hipMemcpyAsync(w.Lam, opt.warm_Lambda, sizeof(double) * qq,
                                    hipMemcpyDeviceToDevice, s));
        } else {
            set_identity(s, q, w.Lam);
        }
        if (opt.warm_Theta) {
            CGGM_HIP(hipMemcpyAsync(w.Th, opt.warm_Theta, sizeof(double) * pq,
                                    hipMemcpyDeviceToDevice, s));
        } else {
            fill(s, pq, 0.0, w.Th);
        }
        CGGM_HIP(hipMemcpyAsync(w.L, w.Lam, sizeof(double) * qq, hipMemcpyDeviceToDevice, s));
        set_int(s, w.flag, 0);
        cholesky_inplace(s, q, w.L, w.flag, w.Wd);
        int hflag = 0;
        CGGM_HIP(hipMemcpyAsync(&hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        CGGM_HIP(hipStreamSynchronize(s));
        if (hflag) fail(CGGM_ENOTPD, "the warm-start Lambda is not positive definite");
        refresh_sigma(c);
        theta_products(c, X);
        started = true;
    }
    SolveOutcome run(double lamL, double lamT, double tol);
    void direction(double lamL, double lamT, double *D_out, double *U_out, double *V_out);
};

// One Lambda direction at the current iterate (the top-of-iteration
// evaluation, the active sets and options.lambda_passes CD passes, in the
// run's precision and schedule at options.split_level) and V = Theta Sigma as
// the Theta step forms it; D, the maintained U = D Sigma and V are copied out
// in FP64.  The iterate is not changed.
void Solver::Impl::direction(double lamL, double lamT, double *D_out, double *U_out,
                             double *V_out) {
    if (!started) fail(CGGM_EINVAL, "direction before start");
    check_lambda(lamL, lamT);
    Ctx c{s, w, lamL, lamT, mixed};
    reduce_dot(s, w.n * q, w.A, w.R, w.partials, w.scal + S_AR);
    gradients(c, X);
    reduce_top_stats(s, p, q, w.Sxy, w.GT, w.Th, lamT, 0, w.partials, w.scal + S_THETA);
    double h[5];
    CGGM_HIP(hipMemcpyAsync(h, w.scal + S_THETA, sizeof(h), hipMemcpyDeviceToHost, s));
    CGGM_HIP(hipStreamSynchronize(s));
    c.theta_density = h[4] / ((double)p * (double)q);   // V as the Theta step forms it
    const Schedule &sch = split_sched(la_split, la_sched, seq ? 0 : opt.split_level);
    for (int pass = 0; pass < opt.lambda_passes; ++pass) run_lambda_sweep(c, sch, nullptr, pass);
    theta_sigma(c);
    const int64_t qq = q * q;
    auto out2d = [&](double *dst, int64_t rows, const double *src64, const float *src32) {
        if (!dst) return;
        if (src32) {
            const int64_t count = rows * q;
            widen2d_kernel<<<nblk(count), BLOCK, 0, s>>>(rows, q, src32, f32_ld(q), dst, q);
            CGGM_LAUNCH_CHECK();
        } else {
            CGGM_HIP(hipMemcpyAsync(dst, src64, sizeof(double) * rows * q, hipMemcpyDeviceToDevice,
                                    s));
        }
    };
    if (D_out)
        CGGM_HIP(hipMemcpyAsync(D_out, w.D, sizeof(double) * qq, hipMemcpyDeviceToDevice, s));
    out2d(U_out, q, w.U, c.f32() ? w.U32 : nullptr);
    out2d(V_out, p, w.V, c.f32() ? w.V32 : nullptr);
    CGGM_HIP(hipStreamSynchronize(s));
}

// Algorithm 1 from the current iterate (Lambda, its factor L, Sigma, Theta,
// A = X Theta and R = A Sigma all current) to the stopping rule.  On return
// the same quantities are current for the returned iterate.
SolveOutcome Solver::Impl::run(double lamL, double lamT, double tol) {
    if (!started) fail(CGGM_EINVAL, "run before start");
    check_lambda(lamL, lamT);
    if (!(tol >= 0.0) || !isfinite(tol)) fail(CGGM_EINVAL, "tol must be finite and >= 0");
    Ctx c{s, w, lamL, lamT, mixed};
    if (opt.graphs && !seq) c.graphs = &graphs;
    // Mixed mode forms V from split-BF16 products while the iterate is far
    // from the optimum and switches to FP64 for the rest of the run once the
    // subgradient falls below MIXED_FP64_BELOW of the stopping scale: the
    // ~1e-6 relative error of V would otherwise bound how far the Theta sweep
    // can reduce the subgradient.
    constexpr double MIXED_FP64_BELOW = 1e-4;
    // The Theta descent guard compares FP64 objectives; after a sweep steered
    // by the split-BF16 V it allows the larger increase that error permits.
    bool swept_mixed = c.mixed;
    const int64_t qq = q * q, pq = p * q;

    // Concurrency of the tiled sweeps: each wave runs as 2^level sub-waves
    // whose tiles see the updates of the earlier sub-waves (Jacobi across the
    // tiles of one sub-wave, exact Gauss-Seidel inside a tile).  With many
    // strongly coupled tiles per wave the concurrent (Jacobi) part can give a
    // poor or even divergent direction, so a direction without descent or
    // without an Armijo step, a Theta sweep that raised f, or a Lambda step
    // the line search had to shrink below SMALL_STEP raises the level; three
    // full steps (three Theta sweeps that pass the guard) in a row lower it
    // again.  The levels start at options.split_level; with
    // options.split_adapt == 0 they stay there and a failing sweep goes
    // straight to one tile per wave.
    constexpr double SMALL_STEP = 0.125;
    const bool adapt = opt.split_adapt != 0;
    int la_level = seq ? 0 : opt.split_level, th_level = la_level, la_good = 0, th_good = 0;
    int status = CGGM_MAXITER, stalled = 0, t = 0, ls_fail_streak = 0;
    double sg_best = INFINITY, f_prev = INFINITY, f_after_ls = INFINITY;
    bool have_phase = false;
    const int trace_first = trace_len;
    int last_trials = 0, last_fallbacks = 0;
    double last_alpha = 0.0, last_delta = 0.0;
    TopStats top{};
    for (t = 0;; ++t) {
        CGGM_HIP(hipEventRecord(ev[0], s));
        // ---- top of the iteration: objective, gradients, screen, stopping
        // statistics (A, R already current), read back in one transfer ------
        auto evaluate = [&] {
            reduce_dot(s, w.n * q, w.A, w.R, w.partials, w.scal + S_AR);
            gradients(c, X);
            reduce_top_stats(s, p, q, w.Sxy, w.GT, w.Th, lamT, 0, w.partials, w.scal + S_THETA);
            reduce_top_stats(s, q, q, w.Syy, w.GL, w.Lam, lamL, 1, w.partials, w.scal + S_LAM);
        };
        reduce_logdet(s, q, w.L, w.partials, w.scal + S_LOGDET);
        evaluate();
        CGGM_HIP(hipEventRecord(ev[1], s));
        top = read_top(c, true);
        c.theta_density = (double)top.nnzT / ((double)p * (double)q);
        kt_theta.collect();                       // the last Theta sweep is done
        // Descent guard: the Theta sweep must not raise f.  A sweep steered by
        // the mixed-precision operands is redone in FP64 at the same level (and
        // the run stays in FP64); a tiled FP64 sweep that raised f is redone
        // with its waves split further, and past MAX_SPLIT_LEVEL one tile per
        // wave (exact block Gauss-Seidel; at q = 20000 about a minute).
        bool th_fired = false;
        while (t > 0 && !seq) {
            if (!(top.f > f_after_ls + F_ROUNDING * std::max(1.0, fabs(f_after_ls)))) break;
            th_fired = true;
            CGGM_HIP(hipMemcpyAsync(w.Th, w.ThOld, sizeof(double) * pq, hipMemcpyDeviceToDevice,
                                    s));
            const Schedule *sch = &th_safe;
            if (swept_mixed) {
                sch = &split_sched(th_split, th_sched, th_level);
            } else if (adapt && th_level < MAX_SPLIT_LEVEL) {
                ++th_level;
                sch = &split_sched(th_split, th_sched, th_level);
            }
            c.mixed = false;
            swept_mixed = false;
            theta_sigma(c);
            for (int pass = 0; pass < opt.theta_passes; ++pass)
                run_theta_sweep(c, *sch, nullptr, pass, &slab);
            ++last_fallbacks;
            theta_products(c, X);
            evaluate();
            CGGM_HIP(hipEventRecord(ev[1], s));
            top = read_top(c, true);
            if (sch == &th_safe) break;
        }
        if (adapt && t > 0 && !th_fired && th_level > 0 && ++th_good >= 3) {
            --th_level;
            th_good = 0;
        }
        if (th_fired) th_good = 0;
        if (opt.trace && trace_len < opt.trace_cap) {
            cggm_trace_entry &te = opt.trace[trace_len++];
            memset(&te, 0, sizeof(te));
            te.iter = t;
            te.f = top.f;
            te.subgrad_l1 = top.subgrad;
            te.l1 = top.l1;
            te.m_Lambda = top.mL;
            te.m_Theta = top.mT;
            te.nnz_Lambda = top.nnzL;
            te.nnz_Theta = top.nnzT;
            te.sweep_split = la_level | (th_level << 8);
            te.t_end_ms = ms_since(t0);
            float ms = 0.f;
            CGGM_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            te.ms_gradient = ms;
            if (t > 0 && trace_len - trace_first >= 2) {
                cggm_trace_entry &pv = opt.trace[trace_len - 2];
                pv.alpha = last_alpha;
                pv.delta = last_delta;
                pv.ls_trials = last_trials;
                pv.sweep_fallbacks = last_fallbacks;
                if (have_phase) {
                    CGGM_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
                    pv.ms_lambda_cd = ms;
                    CGGM_HIP(hipEventElapsedTime(&ms, ev[3], ev[4]));
                    pv.ms_line_search = ms;
                    CGGM_HIP(hipEventElapsedTime(&ms, ev[4], ev[0]));
                    pv.ms_theta_cd = ms;
                }
            }
        }
        last_fallbacks = 0;
        if (c.mixed && top.subgrad < MIXED_FP64_BELOW * top.l1) c.mixed = false;
        if (top.subgrad < tol * top.l1) {
            status = CGGM_OK;
            break;
        }
        if (opt.stall_iters > 0) {
            const bool no_progress = (top.subgrad >= sg_best) &&
                                     (top.f >= f_prev - 1e-15 * fabs(f_prev));
            stalled = no_progress ? stalled + 1 : 0;
            if (stalled >= opt.stall_iters) {
                status = CGGM_STALLED;
                break;
            }
        }
        sg_best = std::min(sg_best, top.subgrad);
        f_prev = top.f;
        if (t >= opt.max_iter) {
            status = CGGM_MAXITER;
            break;
        }

        // ---- Lambda: Newton direction by CD passes, Armijo line search -----
        CGGM_HIP(hipEventRecord(ev[2], s));
        // The direction: lambda_passes CD passes over S_Lambda at schedule
        // `sch`; returns delta = tr(G D) + lamL (|Lambda + D|_1 - |Lambda|_1).
        auto direction = [&](const Schedule &sch, KernelTimer *kt) {
            for (int pass = 0; pass < opt.lambda_passes; ++pass) {
                run_lambda_sweep(c, sch, kt, pass);
                if (kt && pass + 1 < opt.lambda_passes && kt->on()) {
                    // recycle the timing events of this pass
                    CGGM_HIP(hipStreamSynchronize(s));
                    kt->collect();
                }
            }
            reduce_direction(s, q, w.GL, w.Lam, w.D, w.partials, w.scal + S_DIR);
            double hd[2];
            CGGM_HIP(hipMemcpyAsync(hd, w.scal + S_DIR, sizeof(hd), hipMemcpyDeviceToHost, s));
            CGGM_HIP(hipStreamSynchronize(s));
            if (kt) kt->collect();
            return hd[0] + lamL * hd[1];
        };
        // Armijo rule along D (Algorithm 1): the first alpha = 1, beta, ... with
        // Lambda + alpha D positive definite (Cholesky) and f decreased by at
        // least ls_sigma alpha delta; the trial's factor is kept for the swap.
        double alpha = 0.0, f_acc = top.f;
        int trials = 0;
        auto line_search = [&](double delta) {
            transpose(s, w.n, q, w.A, w.At);            // A^T, q x n
            double a = 1.0;
            for (int k = 0; k < opt.max_ls; ++k, a *= opt.ls_beta) {
                ++trials;
                build_trial(s, q, w.Lam, w.D, a, w.Syy, w.LamT, w.partials, w.scal + S_TRIAL);
                CGGM_HIP(hipMemcpyAsync(w.Lt, w.LamT, sizeof(double) * qq,
                                        hipMemcpyDeviceToDevice, s));
                set_int(s, w.flag, 0);
                cholesky_inplace(s, q, w.Lt, w.flag, w.Wdt);
                reduce_logdet(s, q, w.Lt, w.partials, w.scal + S_TLOGDET);
                CGGM_HIP(hipMemcpyAsync(w.Zt, w.At, sizeof(double) * w.n * q,
                                        hipMemcpyDeviceToDevice, s));
                trsm_lower_left(s, q, w.Lt, w.Wdt, w.Zt, w.n, w.n, false);
                reduce_dot(s, q * w.n, w.Zt, w.Zt, w.partials, w.scal + S_ZZ);
                double h[6];
                int hf = 0;
                CGGM_HIP(hipMemcpyAsync(h, w.scal + S_TRIAL, sizeof(h), hipMemcpyDeviceToHost, s));
                CGGM_HIP(hipMemcpyAsync(&hf, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
                CGGM_HIP(hipStreamSynchronize(s));
                const double trS = h[0], l1T = h[1], ld = h[2], bad = h[3], zz = h[4];
                if (hf || bad != 0.0 || !isfinite(zz)) continue;      // not positive definite
                const double fa = -ld + trS + 2.0 * top.sxyT + zz / (double)w.n + lamL * l1T +
                                  lamT * top.l1T;
                if (fa <= top.f + opt.ls_sigma * a * delta +
                              F_ROUNDING * std::max(1.0, fabs(top.f))) {
                    alpha = a;
                    f_acc = fa;
                    return true;
                }
            }
            return false;
        };
        // Descent guard: a direction without descent (delta >= 0), or one for
        // which no Armijo step was found, is redone: a direction from the
        // mixed-precision operands in FP64 at the same level (the run then
        // stays in FP64), a tiled FP64 direction with its waves split further,
        // and past MAX_SPLIT_LEVEL (or at a fixed level) with one tile per
        // wave, whose outcome stands.
        const Schedule *la_sch = &split_sched(la_split, la_sched, la_level);
        double delta = direction(*la_sch, &kt_lambda);
        bool accepted = false;
        for (;;) {
            CGGM_HIP(hipEventRecord(ev[3], s));
            if (delta < 0.0) accepted = line_search(delta);
            if (accepted || seq || la_sch == &la_safe) break;
            if (c.mixed) {
                // same schedule, FP64 operands
            } else if (adapt && la_level < MAX_SPLIT_LEVEL) {
                ++la_level;
                la_good = 0;
                la_sch = &split_sched(la_split, la_sched, la_level);
            } else {
                la_sch = &la_safe;
            }
            c.mixed = false;
            delta = direction(*la_sch, nullptr);
            ++last_fallbacks;
        }
        if (accepted) {
            std::swap(w.Lam, w.LamT);
            std::swap(w.L, w.Lt);
            std::swap(w.Wd, w.Wdt);
            ls_fail_streak = 0;
        } else if (delta < 0.0) {
            if (++ls_fail_streak >= 2) {
                status = CGGM_ELINESEARCH;
                break;
            }
        }
        if (!seq && adapt && accepted) {
            if (alpha < SMALL_STEP && la_level < MAX_SPLIT_LEVEL) {
                ++la_level;
                la_good = 0;
            } else if (alpha < 1.0) {
                la_good = 0;
            } else if (la_level > 0 && ++la_good >= 3) {
                --la_level;
                la_good = 0;
            }
        }
        last_delta = delta;
        f_after_ls = f_acc;
        last_alpha = alpha;
        last_trials = trials;
        refresh_sigma(c);
        CGGM_HIP(hipEventRecord(ev[4], s));
        have_phase = true;

        // ---- Theta: one CD pass on Eq. (7) with Sigma of the new Lambda ----
        CGGM_HIP(hipMemcpyAsync(w.ThOld, w.Th, sizeof(double) * pq, hipMemcpyDeviceToDevice, s));
        swept_mixed = c.mixed;
        theta_sigma(c);                                              // V = Theta Sigma
        for (int pass = 0; pass < opt.theta_passes; ++pass)
            run_theta_sweep(c, split_sched(th_split, th_sched, th_level), &kt_theta, pass,
                            &slab);
        theta_products(c, X);
    }
    SolveOutcome o;
    o.status = status;
    o.iters = t;
    o.f = top.f;
    return o;
}

Solver::Solver(int64_t n, int64_t p, int64_t q, const cggm_options *opt, hipStream_t s,
               int dtype)
    : impl_(new Impl(n, p, q, opt, s, dtype)) {}
Solver::~Solver() = default;
size_t Solver::footprint() const { return impl_->bytes; }
void Solver::allocate() { impl_->allocate(); }
void Solver::bind(void *base) { impl_->bind(base); }
void Solver::load(const void *X, const void *Y) { impl_->load(X, Y); }
void Solver::start() { impl_->start(); }
SolveOutcome Solver::run(double lamL, double lamT, double tol) {
    return impl_->run(lamL, lamT, tol);
}
int Solver::trace_len() const { return impl_->trace_len; }
void Solver::direction(double lamL, double lamT, double *D, double *U, double *V) {
    impl_->direction(lamL, lamT, D, U, V);
}

void Solver::copy_dense(double *Lambda, double *Theta) {
    Impl &m = *impl_;
    if (Lambda)
        CGGM_HIP(hipMemcpyAsync(Lambda, m.w.Lam, sizeof(double) * m.q * m.q,
                                hipMemcpyDeviceToDevice, m.s));
    if (Theta)
        CGGM_HIP(hipMemcpyAsync(Theta, m.w.Th, sizeof(double) * m.p * m.q,
                                hipMemcpyDeviceToDevice, m.s));
}

cggm_result *Solver::make_result(const SolveOutcome &o) {
    Impl &m = *impl_;
    const int64_t qq = m.q * m.q, pq = m.p * m.q;
    auto *res = new ResultImpl();
    std::unique_ptr<ResultImpl> guard(res);
    res->p = m.p;
    res->q = m.q;
    res->iters = o.iters;
    res->f = o.f;
    res->status = o.status;
    CGGM_HIP(hipMalloc(&res->Lam, sizeof(double) * qq));
    CGGM_HIP(hipMalloc(&res->Th, sizeof(double) * pq));
    copy_dense(res->Lam, res->Th);
    to_csr(m.s, m.q, m.q, res->Lam, &res->L_rowptr, &res->L_col, &res->L_val, &res->nnzL);
    to_csr(m.s, m.p, m.q, res->Th, &res->T_rowptr, &res->T_col, &res->T_val, &res->nnzT);
    return reinterpret_cast<cggm_result *>(guard.release());
}

void Solver::finish_kernel_stats() {
    Impl &m = *impl_;
    if (!m.opt.kstats) return;
    CGGM_HIP(hipStreamSynchronize(m.s));
    m.kt_theta.collect();
    unsigned long long h[16];
    CGGM_HIP(hipMemcpyAsync(h, m.w.kctr, sizeof(h), hipMemcpyDeviceToHost, m.s));
    CGGM_HIP(hipStreamSynchronize(m.s));
    cggm_kernel_stats &ks = *m.opt.kstats;
    const KernelTimer *kts[2] = {&m.kt_lambda, &m.kt_theta};
    for (int k = 0; k < 2; ++k) {
        ks.waves[k] = kts[k]->waves;
        ks.tiles[k] = (int64_t)h[8 * k];
        for (int j = 0; j < 3; ++j) {
            ks.ms[k][j] = kts[k]->ms[j];
            ks.bytes[k][j] = (double)h[8 * k + 1 + 2 * j];
            ks.flops[k][j] = (double)h[8 * k + 2 + 2 * j];
        }
    }
}

size_t solve_footprint(int64_t n, int64_t p, int64_t q, const cggm_options *opt, int dtype) {
    Solver sv(n, p, q, opt, nullptr, dtype);
    return sv.footprint();
}

void set_last_error(const std::string &msg) { g_last_error = msg; }
std::string last_error_text() { return g_last_error; }

int combine_status(int acc, int s) {
    if (acc < 0) return acc;
    if (s < 0) return s;
    if (acc == CGGM_MAXITER || s == CGGM_MAXITER) return CGGM_MAXITER;
    return std::max(acc, s);
}

namespace {

int solve_impl(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
               double lamL, double lamT, double tol, cggm_options *opt_in, cggm_result **out,
               hipStream_t s) {
    if (!X || !Y || !out) fail(CGGM_EINVAL, "NULL pointer argument");
    check_sizes(n, p, q);
    check_dtype(dtype);
    check_lambda(lamL, lamT);
    if (!(tol >= 0.0) || !isfinite(tol)) fail(CGGM_EINVAL, "tol must be finite and >= 0");
    Solver sv(n, p, q, opt_in, s, dtype);
    sv.allocate();
    sv.load(X, Y);
    sv.start();
    const SolveOutcome o = sv.run(lamL, lamT, tol);
    sv.finish_kernel_stats();
    if (opt_in) opt_in->trace_len = sv.trace_len();
    *out = sv.make_result(o);
    return o.status;
}

int solve_path_impl(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                    int npath, const double *lamL, const double *lamT, double tol,
                    cggm_options *opt_in, cggm_result **out, hipStream_t s) {
    if (!X || !Y || !out || !lamL || !lamT) fail(CGGM_EINVAL, "NULL pointer argument");
    if (npath < 1) fail(CGGM_EINVAL, "npath must be >= 1");
    check_sizes(n, p, q);
    check_dtype(dtype);
    for (int k = 0; k < npath; ++k) check_lambda(lamL[k], lamT[k]);
    if (!(tol >= 0.0) || !isfinite(tol)) fail(CGGM_EINVAL, "tol must be finite and >= 0");
    Solver sv(n, p, q, opt_in, s, dtype);
    sv.allocate();
    sv.load(X, Y);
    sv.start();
    std::vector<std::unique_ptr<ResultImpl>> res;
    int status = CGGM_OK;
    for (int k = 0; k < npath; ++k) {
        const SolveOutcome o = sv.run(lamL[k], lamT[k], tol);
        res.emplace_back(reinterpret_cast<ResultImpl *>(sv.make_result(o)));
        status = combine_status(status, o.status);
    }
    sv.finish_kernel_stats();
    if (opt_in) opt_in->trace_len = sv.trace_len();
    for (int k = 0; k < npath; ++k) out[k] = reinterpret_cast<cggm_result *>(res[k].release());
    return status;
}

int direction_impl(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                   const double *Lam, const double *Th, double lamL, double lamT,
                   cggm_options *opt_in, double *D, double *U, double *V, hipStream_t s) {
    if (!X || !Y || !Lam || !Th) fail(CGGM_EINVAL, "NULL pointer argument");
    check_sizes(n, p, q);
    check_dtype(dtype);
    check_lambda(lamL, lamT);
    cggm_options opt = checked_options(opt_in);
    opt.warm_Lambda = Lam;
    opt.warm_Theta = Th;
    opt.trace = nullptr;
    opt.kstats = nullptr;
    Solver sv(n, p, q, &opt, s, dtype);
    sv.allocate();
    sv.load(X, Y);
    sv.start();
    sv.direction(lamL, lamT, D, U, V);
    return CGGM_OK;
}

// Tile-edge autotuner: times the outer iterations of a synthetic problem of
// the given shape (X and Y standard normal from a counter-based generator,
// lambda = 0.02, at which the screen is near-dense -- the hard case) for each
// candidate edge, one warm-up iteration and `iters` timed ones from
// Lambda = I, Theta = 0, and returns the fastest by the rule below.  Smaller
// tiles shorten the in-tile Gauss-Seidel chains (R x C dependent steps) and
// put more tiles in a wave; larger ones need fewer waves and launches.
int autotune_impl(int64_t n, int64_t p, int64_t q, const cggm_options *opt_in, int iters,
                  int *tile_out, double *ms_out, hipStream_t s) {
    if (!tile_out) fail(CGGM_EINVAL, "NULL pointer argument");
    check_sizes(n, p, q);
    if (iters < 1 || iters > 50) fail(CGGM_EINVAL, "iters must be in [1, 50]");
    cggm_options base = checked_options(opt_in);
    DeviceBuffer xy;
    if (hipMalloc(&xy.p, sizeof(double) * n * (p + q)) != hipSuccess) {
        (void)hipGetLastError();
        fail(CGGM_ENOMEM, "hipMalloc of the tuner's inputs failed");
    }
    double *X = (double *)xy.p, *Y = X + n * p;
    normal_kernel<<<nblk(n * (p + q)), BLOCK, 0, s>>>(n * (p + q), 0x5eedull, X);
    CGGM_LAUNCH_CHECK();
    // Each candidate is timed twice, in the order 64, 32, 16, 16, 32, 64 (so
    // that a drift of the device's speed during the tuning does not favour
    // one edge), and keeps its shorter time; the default edge 64 stays unless
    // a smaller one is at least 5% faster.
    const int cand[3] = {16, 32, 64};
    double best_of[3] = {INFINITY, INFINITY, INFINITY};
    const int order[6] = {2, 1, 0, 0, 1, 2};
    for (int step = 0; step < 6; ++step) {
        const int k = order[step];
        cggm_options o = base;
        o.tile = cand[k];
        o.stall_iters = 0;
        o.max_iter = iters + 1;
        o.warm_Lambda = o.warm_Theta = nullptr;
        o.kstats = nullptr;
        std::vector<cggm_trace_entry> tr(iters + 2);
        o.trace = tr.data();
        o.trace_cap = iters + 2;
        Solver sv(n, p, q, &o, s, CGGM_F64);
        sv.allocate();
        sv.load(X, Y);
        sv.start();
        (void)sv.run(0.02, 0.02, 0.0);
        const int len = sv.trace_len();
        double ms = INFINITY;
        if (len >= 2) ms = (tr[len - 1].t_end_ms - tr[1].t_end_ms) / std::max(1, len - 2);
        if (len == 2) ms = tr[1].t_end_ms - tr[0].t_end_ms;
        best_of[k] = std::min(best_of[k], ms);
    }
    int best = 2;
    for (int k = 1; k >= 0; --k)
        if (best_of[k] < 0.95 * best_of[best]) best = k;
    if (ms_out)
        for (int k = 0; k < 3; ++k) ms_out[k] = best_of[k];
    *tile_out = cand[best];
    return CGGM_OK;
}

// ------------------------------------------------------- objective/gradient --
// Workspace for the standalone evaluations.
struct EvalWork {
    double *A, *R, *At, *L, *Wd, *Sig, *Psi, *Work, *YL, *partials, *scal;
    int *flag;
    double *X64 = nullptr, *Y64 = nullptr;   // FP64 copies of FP32 inputs
};

// The objective uses A, At, L, Wd, YL and the reduction scratch; the gradient
// A, R, L, Wd, Sig, Psi, Work and the reduction scratch.
void eval_layout(Arena &a, EvalWork &e, int64_t n, int64_t p, int64_t q, bool gradient,
                 int dtype) {
    e.A = a.take<double>(n * q);
    e.R = gradient ? a.take<double>(n * q) : nullptr;
    e.At = gradient ? nullptr : a.take<double>(n * q);
    e.L = a.take<double>(q * q);
    e.Wd = a.take<double>(diag_inv_count(q));
    e.Sig = gradient ? a.take<double>(q * q) : nullptr;
    e.Psi = gradient ? a.take<double>(q * q) : nullptr;
    e.Work = gradient ? a.take<double>(q * q) : nullptr;
    e.YL = gradient ? nullptr : a.take<double>(n * q);
    e.partials = a.take<double>(REDUCE_BLOCKS * 8);
    e.scal = a.take<double>(NSCAL);
    e.flag = a.take<int>(4);
    if (dtype == CGGM_F32) {
        e.X64 = a.take<double>(n * p);
        e.Y64 = a.take<double>(n * q);
    }
}

// f of Eq. (1) at dense (Lam, Th) with the evaluation workspace `e` (laid out
// for the objective); Lam must be positive definite (else CGGM_ENOTPD).
// f = -log det L + tr(Syy Lam) + 2 <Sxy, Theta> + |L^{-1} (X Theta)^T|_F^2 / n
//     + penalties, with tr(Syy Lam) = <Y, Y Lam> / n, <Sxy, Theta> = <Y, X Theta> / n.
double objective_core(const double *X, const double *Y, int64_t n, int64_t p, int64_t q,
                      const double *Lam, const double *Th, double lamL, double lamT,
                      const EvalWork &e, hipStream_t s) {
    gemm(s, false, false, n, q, p, 1.0, X, p, Th, q, 0.0, e.A, q);
    CGGM_HIP(hipMemcpyAsync(e.L, Lam, sizeof(double) * q * q, hipMemcpyDeviceToDevice, s));
    set_int(s, e.flag, 0);
    cholesky_inplace(s, q, e.L, e.flag, e.Wd);
    reduce_logdet(s, q, e.L, e.partials, e.scal + 0);
    transpose(s, n, q, e.A, e.At);
    trsm_lower_left(s, q, e.L, e.Wd, e.At, n, n, false);
    reduce_dot(s, q * n, e.At, e.At, e.partials, e.scal + 2);
    gemm(s, false, false, n, q, q, 1.0, Y, q, Lam, q, 0.0, e.YL, q);
    reduce_dot(s, n * q, Y, e.YL, e.partials, e.scal + 3);
    reduce_dot(s, n * q, Y, e.A, e.partials, e.scal + 4);
    // l1 norms through the top-stats reduction (W = P, G unused)
    reduce_top_stats(s, q, q, Lam, Lam, Lam, 0.0, 0, e.partials, e.scal + 5);
    reduce_top_stats(s, p, q, Th, Th, Th, 0.0, 0, e.partials, e.scal + 10);
    double h[16];
    int hf = 0;
    CGGM_HIP(hipMemcpyAsync(h, e.scal, sizeof(h), hipMemcpyDeviceToHost, s));
    CGGM_HIP(hipMemcpyAsync(&hf, e.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    CGGM_HIP(hipStreamSynchronize(s));
    if (hf || h[1] != 0.0) fail(CGGM_ENOTPD, "Lambda is not positive definite");
    const double inv_n = 1.0 / (double)n;
    return -h[0] + h[3] * inv_n + 2.0 * h[4] * inv_n + h[2] * inv_n + lamL * h[6] + lamT * h[11];
}

void check_objective_args(const void *X, const void *Y, int64_t n, int64_t p, int64_t q,
                          int dtype, const double *Lam, const double *Th, double lamL,
                          double lamT, double *f_out) {
    if (!X || !Y || !Lam || !Th || !f_out) fail(CGGM_EINVAL, "NULL pointer argument");
    check_sizes(n, p, q);
    check_dtype(dtype);
    check_lambda(lamL, lamT);
}

int objective_impl(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                   const double *Lam, const double *Th, double lamL, double lamT, double *f_out,
                   hipStream_t s) {
    check_objective_args(X, Y, n, p, q, dtype, Lam, Th, lamL, lamT, f_out);
    Arena sizer;
    sizer.measure = true;
    EvalWork e;
    eval_layout(sizer, e, n, p, q, false, dtype);
    DeviceBuffer buf;
    if (hipMalloc(&buf.p, sizer.used) != hipSuccess) {
        (void)hipGetLastError();
        fail(CGGM_ENOMEM, "hipMalloc failed");
    }
    Arena arena;
    arena.base = (char *)buf.p;
    eval_layout(arena, e, n, p, q, false, dtype);
    const auto [X64, Y64] = fp64_inputs(s, dtype, n, p, q, X, Y, e.X64, e.Y64);
    *f_out = objective_core(X64, Y64, n, p, q, Lam, Th, lamL, lamT, e, s);
    return CGGM_OK;
}

// Device address of the allocation-free entry point's scratch array on the
// current device, looked up once per device (with that device current) and
// kept: each device holds its own copy of the array at its own address, and
// the array's name in host code is only a host-side stand-in.
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_addr;

void *scratch_on_current_device() {
    int dev = 0;
    CGGM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !ptr)
            fail(CGGM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(err));
        g_scratch_addr[dev] = ptr;
    }
    return g_scratch_addr[dev];
}

int objective_noalloc_impl(const void *X, const void *Y, int64_t n, int64_t p, int64_t q,
                           int dtype, const double *Lam, const double *Th, double lamL,
                           double lamT, double *f_out, hipStream_t s) {
    check_objective_args(X, Y, n, p, q, dtype, Lam, Th, lamL, lamT, f_out);
    Arena sizer;
    sizer.measure = true;
    EvalWork e;
    eval_layout(sizer, e, n, p, q, false, dtype);
    if (sizer.used > (size_t)CGGM_NOALLOC_SCRATCH_BYTES)
        fail(CGGM_ECAPACITY, "cggm_objective_noalloc: the workspace of this shape (" +
                                 std::to_string(sizer.used) + " bytes) exceeds the " +
                                 std::to_string((size_t)CGGM_NOALLOC_SCRATCH_BYTES) +
                                 "-byte static scratch");
    Arena arena;
    arena.base = (char *)scratch_on_current_device();
    eval_layout(arena, e, n, p, q, false, dtype);
    const auto [X64, Y64] = fp64_inputs(s, dtype, n, p, q, X, Y, e.X64, e.Y64);
    *f_out = objective_core(X64, Y64, n, p, q, Lam, Th, lamL, lamT, e, s);
    return CGGM_OK;
}

int gradient_impl(const void *X_in, const void *Y_in, int64_t n, int64_t p, int64_t q,
                  int dtype, const double *Lam, const double *Th, double *GL, double *GT,
                  hipStream_t s) {
    if (!X_in || !Y_in || !Lam || !Th || !GL || !GT) fail(CGGM_EINVAL, "NULL pointer argument");
    check_sizes(n, p, q);
    check_dtype(dtype);
    Arena sizer;
    sizer.measure = true;
    EvalWork e;
    eval_layout(sizer, e, n, p, q, true, dtype);
    DeviceBuffer buf;
    if (hipMalloc(&buf.p, sizer.used) != hipSuccess) {
        (void)hipGetLastError();
        fail(CGGM_ENOMEM, "hipMalloc failed");
    }
    Arena arena;
    arena.base = (char *)buf.p;
    eval_layout(arena, e, n, p, q, true, dtype);
    const auto [X, Y] = fp64_inputs(s, dtype, n, p, q, X_in, Y_in, e.X64, e.Y64);
    const double inv_n = 1.0 / (double)n;
    CGGM_HIP(hipMemcpyAsync(e.L, Lam, sizeof(double) * q * q, hipMemcpyDeviceToDevice, s));
    set_int(s, e.flag, 0);
    cholesky_inplace(s, q, e.L, e.flag, e.Wd);
    reduce_logdet(s, q, e.L, e.partials, e.scal);
    int hf = 0;
    double h[2];
    CGGM_HIP(hipMemcpyAsync(&hf, e.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    CGGM_HIP(hipMemcpyAsync(h, e.scal, sizeof(h), hipMemcpyDeviceToHost, s));
    CGGM_HIP(hipStreamSynchronize(s));
    if (hf || h[1] != 0.0) fail(CGGM_ENOTPD, "Lambda is not positive definite");
    spd_inverse_from_cholesky(s, q, e.L, e.Wd, e.Work, e.Sig);
    gemm(s, false, false, n, q, p, 1.0, X, p, Th, q, 0.0, e.A, q);        // A = X Theta
    gemm(s, false, false, n, q, q, 1.0, e.A, q, e.Sig, q, 0.0, e.R, q);   // R = A Sigma
    gemm(s, true, false, q, q, n, inv_n, e.R, q, e.R, q, 0.0, e.Psi, q, UPLO_LOWER);
    symmetrize_from_lower(s, q, e.Psi);
    gemm(s, true, false, q, q, n, inv_n, Y, q, Y, q, 0.0, e.Work, q, UPLO_LOWER);   // Syy
    symmetrize_from_lower(s, q, e.Work);
    assemble_lambda_gradient(s, q, e.Work, e.Sig, e.Psi, GL, e.Work);   // SP unused
    // G_Theta = (2/n) X^T (Y + R)
    add_kernel<<<nblk(n * q), BLOCK, 0, s>>>(n * q, Y, e.R);
    CGGM_LAUNCH_CHECK();
    gemm(s, true, false, p, q, n, 2.0 * inv_n, X, p, e.R, q, 0.0, GT, q);
    CGGM_HIP(hipStreamSynchronize(s));
    return CGGM_OK;
}

}  // namespace
}  // namespace cggm

// ================================================================= C ABI =====
using namespace cggm;

extern "C" {

void cggm_default_options(cggm_options *opt) {
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->max_iter = 500;
    opt->max_ls = 30;
    opt->ls_beta = 0.5;
    opt->ls_sigma = 1e-3;
    opt->stall_iters = 3;
    opt->sweep = CGGM_SWEEP_TILED;
    opt->tile = 0;
    opt->lambda_passes = 0;
    opt->precision = CGGM_PRECISION_FP64;
    opt->mixed_min_q = 4096;
    opt->theta_passes = 1;
    opt->split_level = 0;
    opt->split_adapt = 1;
    opt->blockwise = 0;
    opt->sxx_cache_bytes = 0;
    opt->graphs = 0;
}

size_t cggm_solve_workspace_bytes(int64_t n, int64_t p, int64_t q) {
    return cggm_workspace_bytes(n, p, q, nullptr);
}

size_t cggm_workspace_bytes(int64_t n, int64_t p, int64_t q, const cggm_options *opt) {
    size_t bytes = 0;
    const int st = guarded([&] {
        bytes = solve_footprint(n, p, q, opt, CGGM_F64);
        return CGGM_OK;
    });
    return st == CGGM_OK ? bytes : 0;
}

int cggm_solve(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
               double lamL, double lamT, double tol, cggm_options *opt, cggm_result **out,
               void *stream) {
    return guarded([&] {
        return solve_impl(X, Y, n, p, q, dtype, lamL, lamT, tol, opt, out, (hipStream_t)stream);
    });
}

int cggm_solve_path(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                    int npath, const double *lamL, const double *lamT, double tol,
                    cggm_options *opt, cggm_result **out, void *stream) {
    return guarded([&] {
        return solve_path_impl(X, Y, n, p, q, dtype, npath, lamL, lamT, tol, opt, out,
                               (hipStream_t)stream);
    });
}

int cggm_result_info(const cggm_result *res, int64_t *nnz_Lambda, int64_t *nnz_Theta,
                     int *iters, double *f, int *status) {
    return guarded([&] {
        if (!res) fail(CGGM_EINVAL, "NULL result");
        const auto *r = reinterpret_cast<const ResultImpl *>(res);
        if (nnz_Lambda) *nnz_Lambda = r->nnzL;
        if (nnz_Theta) *nnz_Theta = r->nnzT;
        if (iters) *iters = r->iters;
        if (f) *f = r->f;
        if (status) *status = r->status;
        return CGGM_OK;
    });
}

int cggm_result_copy(const cggm_result *res, int64_t *L_rowptr, int32_t *L_col, double *L_val,
                     int64_t *T_rowptr, int32_t *T_col, double *T_val, int to_host) {
    return guarded([&] {
        if (!res) fail(CGGM_EINVAL, "NULL result");
        const auto *r = reinterpret_cast<const ResultImpl *>(res);
        const hipMemcpyKind k = to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        auto cp = [&](void *dst, const void *src, size_t bytes) {
            if (dst && bytes) CGGM_HIP(hipMemcpy(dst, src, bytes, k));
        };
        cp(L_rowptr, r->L_rowptr, sizeof(int64_t) * (r->q + 1));
        cp(L_col, r->L_col, sizeof(int32_t) * r->nnzL);
        cp(L_val, r->L_val, sizeof(double) * r->nnzL);
        cp(T_rowptr, r->T_rowptr, sizeof(int64_t) * (r->p + 1));
        cp(T_col, r->T_col, sizeof(int32_t) * r->nnzT);
        cp(T_val, r->T_val, sizeof(double) * r->nnzT);
        return CGGM_OK;
    });
}

int cggm_result_dense(const cggm_result *res, double *Lambda, double *Theta, int to_host) {
    return guarded([&] {
        if (!res) fail(CGGM_EINVAL, "NULL result");
        const auto *r = reinterpret_cast<const ResultImpl *>(res);
        const hipMemcpyKind k = to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        if (Lambda) CGGM_HIP(hipMemcpy(Lambda, r->Lam, sizeof(double) * r->q * r->q, k));
        if (Theta) CGGM_HIP(hipMemcpy(Theta, r->Th, sizeof(double) * r->p * r->q, k));
        return CGGM_OK;
    });
}

void cggm_result_free(cggm_result *res) { delete reinterpret_cast<ResultImpl *>(res); }

int cggm_objective(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                   const double *Lambda, const double *Theta, double lamL, double lamT,
                   double *f_out, void *stream) {
    return guarded([&] {
        return objective_impl(X, Y, n, p, q, dtype, Lambda, Theta, lamL, lamT, f_out,
                              (hipStream_t)stream);
    });
}

int cggm_objective_noalloc(const void *X, const void *Y, int64_t n, int64_t p, int64_t q,
                           int dtype, const double *Lambda, const double *Theta, double lamL,
                           double lamT, double *f_out, void *stream) {
    return guarded([&] {
        return objective_noalloc_impl(X, Y, n, p, q, dtype, Lambda, Theta, lamL, lamT, f_out,
                                      (hipStream_t)stream);
    });
}

int cggm_autotune_tile(int64_t n, int64_t p, int64_t q, const cggm_options *opt, int iters,
                       int *tile, double *ms, void *stream) {
    return guarded([&] {
        return autotune_impl(n, p, q, opt, iters, tile, ms, (hipStream_t)stream);
    });
}

int cggm_lambda_direction(const void *X, const void *Y, int64_t n, int64_t p, int64_t q,
                          int dtype, const double *Lambda, const double *Theta, double lamL,
                          double lamT, const cggm_options *opt, double *D, double *U,
                          double *V, void *stream) {
    return guarded([&] {
        cggm_options o;
        cggm_default_options(&o);
        if (opt) o = *opt;
        return direction_impl(X, Y, n, p, q, dtype, Lambda, Theta, lamL, lamT, &o, D, U, V,
                              (hipStream_t)stream);
    });
}

int cggm_gradient(const void *X, const void *Y, int64_t n, int64_t p, int64_t q, int dtype,
                  const double *Lambda, const double *Theta, double *G_Lambda, double *G_Theta,
                  void *stream) {
    return guarded([&] {
        return gradient_impl(X, Y, n, p, q, dtype, Lambda, Theta, G_Lambda, G_Theta,
                             (hipStream_t)stream);
    });
}

const char *cggm_status_string(int status) {
    switch (status) {
        case CGGM_OK: return "ok";
        case CGGM_MAXITER: return "iteration cap reached";
        case CGGM_STALLED: return "stopped at the rounding floor before the stopping rule";
        case CGGM_EINVAL: return "invalid argument";
        case CGGM_ENOTPD: return "Lambda is not positive definite";
        case CGGM_ELINESEARCH: return "line search found no Armijo step";
        case CGGM_ENOMEM: return "out of device memory or over the workspace budget";
        case CGGM_EHIP: return "HIP runtime error";
        case CGGM_ECAPACITY:
            return "problem larger than the device memory the call may use (server pool or "
                   "static scratch)";
        default: return "unknown status";
    }
}

const char *cggm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
