// solver.hpp -- one CGGM problem resident on the device: the host engine of
// Algorithm 1 shared by the solve entry points (engine.hip) and the request
// server (serve.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <new>
#include <string>

#include "cggm.h"
#include "internal.hpp"

namespace cggm {

struct SolveOutcome {
    int status = CGGM_OK;   // CGGM_OK, CGGM_MAXITER, CGGM_STALLED or CGGM_ELINESEARCH
    int iters = 0;          // outer iterations of this run
    double f = 0.0;         // objective at the returned iterate
};

// Lifecycle: construct (validates sizes and options, sizes the workspace)
// -> allocate() or bind() -> load(X, Y) -> start() -> run() one or more times.
// Each run() continues from the iterate the previous one returned, so a
// sequence of runs over decreasing penalties is a warm-started path.  All
// device work is ordered on the stream given at construction; run() returns
// with that stream idle.
class Solver {
  public:
    // dtype: CGGM_F64 or CGGM_F32 inputs X, Y (FP32 ones are widened to FP64
    // copies in the workspace at load()).
    Solver(int64_t n, int64_t p, int64_t q, const cggm_options *opt, hipStream_t s,
           int dtype = CGGM_F64);
    ~Solver();
    Solver(const Solver &) = delete;
    Solver &operator=(const Solver &) = delete;

    size_t footprint() const;            // device bytes of the workspace
    void allocate();                     // hipMalloc the workspace (budget checked)
    void bind(void *base);               // use caller memory of footprint() bytes
    void load(const void *X, const void *Y);       // finite check, statistics
    void start();                        // Lambda = I / warm start, Theta = 0 / warm start
    SolveOutcome run(double lamL, double lamT, double tol);
    // Current Lambda (q x q) and Theta (p x q) into device buffers (NULL skips).
    void copy_dense(double *Lambda, double *Theta);
    // A result handle of the current iterate (dense copies and CSR).
    cggm_result *make_result(const SolveOutcome &o);
    int trace_len() const;
    // One Lambda direction at the current iterate and V = Theta Sigma, copied
    // to device buffers (NULL skips): D, U = D Sigma (q x q), V (p x q).
    void direction(double lamL, double lamT, double *D, double *U, double *V);
    void finish_kernel_stats();          // fills options.kstats if given

  private:
    struct Impl;
    std::unique_ptr<Impl> impl_;
};

// Workspace bytes of a solve of this shape with these options (NULL = defaults).
size_t solve_footprint(int64_t n, int64_t p, int64_t q, const cggm_options *opt,
                       int dtype = CGGM_F64);

// Thread-local message of the last failing C-ABI call.
void set_last_error(const std::string &msg);
std::string last_error_text();

// Worst status over the points of a path: the first error, else CGGM_MAXITER
// if any point reached the cap, else CGGM_STALLED if any point stopped at the
// rounding floor, else CGGM_OK.
int combine_status(int acc, int s);

// Runs f, turning exceptions into status codes and the thread's last error.
template <class F>
int guarded(F f) {
    try {
        set_last_error(std::string());
        return f();
    } catch (const Failure &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return CGGM_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return CGGM_EHIP;
    }
}

}  // namespace cggm
