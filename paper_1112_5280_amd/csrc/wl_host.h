// wl_host.h -- host-side drivers of libwilson.so (not installed): the Krylov
// solvers, batched and multi-problem solves, and the solve server. Kernels do
// not include this header.
#pragma once

#include "wl_internal.h"

namespace wl {

// While a thread holds one of these, launches on it use recorded or default
// launch shapes and never time candidates (no events are created).
struct TuningSuspended {
    TuningSuspended();
    ~TuningSuspended();
    TuningSuspended(const TuningSuspended &) = delete;
    TuningSuspended &operator=(const TuningSuspended &) = delete;
};

// packed -> canonical complex128 gauge field (wl_blas.hip)
hipError_t launch_unpack_gauge(const Geom &g, int prec, bool link12, const void *packed,
                               void *canon, hipStream_t s);

// ---- pure gauge (wl_gauge.hip): the canonical complex128 field, or (packed)
// the packed FP64 18-real field --------------------------------------------
hipError_t launch_heatbath_field(const Geom &g, void *field, bool packed, double beta,
                                 int nsweeps, uint32_t sweep0, uint32_t seed, hipStream_t s);
hipError_t launch_plaquette_field(const Geom &g, const void *field, bool packed, double *out,
                                  void *work, hipStream_t s);

// ---- solvers ---------------------------------------------------------------
size_t workspace_bytes(const Geom &g, uint32_t flags);

struct SolveIn {
    const void *gauge, *b;
    void *x;
    Geom g;
    double kappa;
    double mu = 0.0;   // twisted mass (single solves only)
    Phases ph;
    double tol;
    int maxiter;
    uint32_t flags;
    void *work;
    hipStream_t s;
    // batches of independent problems (one lattice size): per-RHS gauge
    // fields (device table) and hopping parameters (host array)
    const void *const *gtab = nullptr;
    const double *kappas = nullptr;
    const void *const *gauges_host = nullptr;   // the gtab entries, readable on the host
    bool own_stream = false;   // `s` belongs to the library: capture on it directly
    bool no_alloc = false;     // read status into plain host memory, no tuning runs
};

int run_solver(bool bicg, const SolveIn &in, wl_solve_stats *st, std::string *why);

// batched CG (FP64, full or even-odd): nrhs fields of b and x, st[nrhs]
// (own_gauges: each RHS has its own gauge field, so a mixed solve keeps one
// low-precision copy per RHS)
size_t workspace_bytes_batch(const Geom &g, uint32_t flags, int nrhs, bool own_gauges = false);
int run_cg_batch(const SolveIn &in, int nrhs, wl_solve_stats *st, std::string *why);

// m problems of one lattice size (own gauge field and kappa each) as one
// batched CG on stream s, in problem_group_bytes(g, flags, m) bytes of work
size_t problem_group_bytes(const Geom &g, uint32_t flags, int m);
int run_problem_group(const wl_problem *const *p, int m, const Geom &g, const Phases &ph,
                      double tol, int maxiter, uint32_t flags, void *work, hipStream_t s,
                      wl_solve_stats *st, std::string *why);

// independent problems of several lattice sizes, solved concurrently
size_t problems_workspace_bytes(const wl_problem *p, int n, uint32_t flags);
int run_problems(const wl_problem *p, int n, const Phases &ph, double tol, int maxiter,
                 uint32_t flags, void *work, hipStream_t caller, wl_solve_stats *st,
                 std::string *why);

// the solve server (wl_server.hip); wl_server itself is the opaque C type
int server_create(const wl_server_config &cfg, const Phases &ph, wl_server **out, std::string *why);
int server_submit(wl_server *s, const wl_problem &p, const Geom &g, uint64_t *ticket,
                  std::string *why);
int server_wait(wl_server *s, uint64_t ticket, wl_solve_stats *st, wl_request_times *t,
                std::string *why);
int server_next(wl_server *s, uint64_t *ticket, wl_solve_stats *st, wl_request_times *t,
                std::string *why);
int server_pending(wl_server *s);
int server_destroy(wl_server *s);

}  // namespace wl
