// wl_api.hip -- the extern "C" boundary of libwilson.so (declared in
// include/wilson.h): argument validation, error reporting and dispatch to the
// launchers and solver drivers. No exception crosses this boundary.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "wl_host.h"

namespace wl {


bool make_geom(const int32_t dims[4], Geom *g, std::string *why) {
    if (!dims) {
        *why = "dims is NULL";
        return false;
    }
    long v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 2 || (dims[mu] & 1)) {
            *why = "every lattice extent must be even and >= 2 (got dims[" + std::to_string(mu) +
                   "] = " + std::to_string(dims[mu]) + ")";
            return false;
        }
        v *= dims[mu];
        g->L[mu] = dims[mu];
    }
    // 36 link chunks per parity block must stay addressable with 32-bit offsets
    if (v / 2 * 36 >= (1L << 31) - 64 * 36) {
        *why = "lattice too large: a parity block's link chunks overflow 32-bit offsets (V = " +
               std::to_string(v) + ")";
        return false;
    }
    g->Lxh = dims[0] / 2;
    g->Vh = int(v / 2);
    g->S = (g->Vh + 63) / 64 * 64;
    g->bpp = (g->Vh + kBlock - 1) / kBlock;
    return true;
}

static size_t complex_bytes(int prec) { return prec == WL_F64 ? 16 : prec == WL_F32 ? 8 : 4; }

size_t spinor_block_bytes(const Geom &g, int prec) {
    // FP16 blocks end with one FP32 scale per site
    return size_t(g.S) * (12 * complex_bytes(prec) + (prec == WL_F16S ? 4 : 0));
}

size_t gauge_bytes(const Geom &g, int prec, bool link12) {
    return size_t(2) * 4 * (link12 ? 6 : 9) * complex_bytes(prec) * size_t(g.S);
}

}  // namespace wl

using namespace wl;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

constexpr uint32_t kKnownFlags = WL_PREC_MASK | WL_LINK12 | WL_DAG | WL_HOP | WL_EO | WL_MIXED | WL_GRAPH |
                                 WL_X0;

bool get_prec(uint32_t flags, int *prec, std::string *why) {
    const uint32_t p = flags & WL_PREC_MASK;
    if (p != WL_F64 && p != WL_F32 && p != WL_F16S) {
        *why = "unsupported precision flag";
        return false;
    }
    *prec = int(p);
    return true;
}

bool get_phases(const double *phases, Phases *ph, std::string *why) {
    if (!phases) {
        *why = "phases is NULL";
        return false;
    }
    for (int mu = 0; mu < 4; ++mu) {
        const double re = phases[2 * mu], im = phases[2 * mu + 1];
        if (!std::isfinite(re) || !std::isfinite(im) || std::fabs(std::hypot(re, im) - 1.0) > 1e-12) {
            *why = "boundary phase " + std::to_string(mu) + " is not of unit modulus";
            return false;
        }
        ph->re[mu] = re;
        ph->im[mu] = im;
    }
    return true;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(WL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" {

const char *wl_version(void) { return "wilson-mi355x 0.1 (gfx950)"; }

const char *wl_last_error(void) { return g_last_error.c_str(); }

size_t wl_spinor_bytes(const int32_t dims[4], uint32_t flags, int32_t nparity) {
    Geom g;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why) || nparity < 1 || nparity > 2)
        return 0;
    return spinor_block_bytes(g, prec) * size_t(nparity);
}

size_t wl_gauge_bytes(const int32_t dims[4], uint32_t flags) {
    Geom g;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why)) return 0;
    return gauge_bytes(g, prec, flags & WL_LINK12);
}

int wl_pack_gauge(const void *canon, void *packed, const int32_t dims[4], uint32_t flags,
                  void *stream) {
    Geom g;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why)) return fail(WL_EINVAL, why);
    if (!canon || !packed) return fail(WL_EINVAL, "NULL buffer");
    if (canon == packed) return fail(WL_EINVAL, "canon and packed alias");
    const hipError_t e = launch_pack_gauge(g, prec, flags & WL_LINK12, canon, packed,
                                           static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_pack_gauge");
}

int wl_pack_spinor(const void *canon, void *packed, const int32_t dims[4], uint32_t flags,
                   void *stream) {
    Geom g;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why)) return fail(WL_EINVAL, why);
    if (!canon || !packed) return fail(WL_EINVAL, "NULL buffer");
    if (canon == packed) return fail(WL_EINVAL, "canon and packed alias");
    const hipError_t e = launch_pack_spinor(g, prec, canon, packed, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_pack_spinor");
}

int wl_unpack_gauge(const void *packed, void *canon, const int32_t dims[4], uint32_t flags,
                    void *stream) {
    Geom g;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why)) return fail(WL_EINVAL, why);
    if (!canon || !packed) return fail(WL_EINVAL, "NULL buffer");
    if (canon == packed) return fail(WL_EINVAL, "canon and packed alias");
    const hipError_t e = launch_unpack_gauge(g, prec, flags & WL_LINK12, packed, canon,
                                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_unpack_gauge");
}

int wl_unpack_spinor(const void *packed, void *canon, const int32_t dims[4], uint32_t flags,
                     void *stream) {
    Geom g;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why)) return fail(WL_EINVAL, why);
    if (!canon || !packed) return fail(WL_EINVAL, "NULL buffer");
    if (canon == packed) return fail(WL_EINVAL, "canon and packed alias");
    const hipError_t e = launch_unpack_spinor(g, prec, packed, canon,
                                              static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_unpack_spinor");
}

int wilson_dslash(const void *gauge, const void *in, void *out, const int32_t dims[4],
                  double kappa, const double phases[8], uint32_t flags, void *stream) {
    return wilson_dslash_tm(gauge, in, out, dims, kappa, 0.0, phases, flags, stream);
}

int wilson_dslash_tm(const void *gauge, const void *in, void *out, const int32_t dims[4],
                     double kappa, double mu, const double phases[8], uint32_t flags,
                     void *stream) {
    Geom g;
    Phases ph;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why) ||
        !get_phases(phases, &ph, &why))
        return fail(WL_EINVAL, why);
    if (!gauge || !in || !out) return fail(WL_EINVAL, "NULL buffer");
    if (in == out) return fail(WL_EINVAL, "in and out alias");
    if (!std::isfinite(kappa)) return fail(WL_EINVAL, "kappa is not finite");
    if (!std::isfinite(mu)) return fail(WL_EINVAL, "mu is not finite");
    if (flags & ~kKnownFlags) return fail(WL_EINVAL, "unknown flag bits");
    const size_t blk = spinor_block_bytes(g, prec);
    HopCall c{};
    c.gauge = gauge;
    c.in[0] = in;
    c.in[1] = static_cast<const char *>(in) + blk;
    c.out[0] = out;
    c.out[1] = static_cast<char *>(out) + blk;
    c.dag = flags & WL_DAG;
    if (!(flags & WL_HOP)) {
        c.xs[0] = c.in[0];
        c.xs[1] = c.in[1];
        c.c = -kappa;
        // twisted mass: (1 + 2 i kappa mu g5) in - kappa D in; adjoint -mu
        const double tw = 2.0 * kappa * mu;
        if (tw != 0.0) c.tx = c.dag ? -tw : tw;
    } else {
        c.c = 1.0;
    }
    c.first_par = 0;
    c.npar = 2;
    const hipError_t e = launch_hop(g, prec, flags & WL_LINK12, ph, c,
                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wilson_dslash");
}

int wilson_dslash_eo(const void *gauge, const void *in, void *out, const int32_t dims[4],
                     double kappa, const double phases[8], int32_t out_parity, uint32_t flags,
                     void *stream) {
    return wilson_dslash_eo_tm(gauge, in, out, dims, kappa, 0.0, phases, out_parity, flags,
                               stream);
}

int wilson_dslash_eo_tm(const void *gauge, const void *in, void *out, const int32_t dims[4],
                        double kappa, double mu, const double phases[8], int32_t out_parity,
                        uint32_t flags, void *stream) {
    Geom g;
    Phases ph;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why) ||
        !get_phases(phases, &ph, &why))
        return fail(WL_EINVAL, why);
    if (!gauge || !in || !out) return fail(WL_EINVAL, "NULL buffer");
    if (in == out) return fail(WL_EINVAL, "in and out alias");
    if (out_parity != 0 && out_parity != 1) return fail(WL_EINVAL, "out_parity must be 0 or 1");
    if (!std::isfinite(kappa)) return fail(WL_EINVAL, "kappa is not finite");
    if (!std::isfinite(mu)) return fail(WL_EINVAL, "mu is not finite");
    const double tw = 2.0 * kappa * mu;   // twist of A = 1 + i tw g5
    if (flags & ~kKnownFlags) return fail(WL_EINVAL, "unknown flag bits");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int p = out_parity, q = 1 - out_parity;
    const bool dag = flags & WL_DAG;
    if (flags & WL_HOP) {
        HopCall c{};
        c.gauge = gauge;
        c.in[q] = in;
        c.out[p] = out;
        c.first_par = p;
        c.npar = 1;
        c.c = 1.0;
        c.dag = dag;
        const hipError_t e = launch_hop(g, prec, flags & WL_LINK12, ph, c, s);
        return e == hipSuccess ? WL_OK : hip_fail(e, "wilson_dslash_eo");
    }
    // Schur complement: tmp_q = D_{q,p} in; out_p = in - kappa^2 D_{p,q} tmp_q.
    // `out` is a full field here: its parity-q block holds the intermediate,
    // so the call needs no scratch of its own.
    const size_t blk = spinor_block_bytes(g, prec);
    void *outp = static_cast<char *>(out) + size_t(p) * blk;
    void *tmp = static_cast<char *>(out) + size_t(q) * blk;
    {
        const char *ib = static_cast<const char *>(in), *ob = static_cast<const char *>(out);
        if (ib < ob + 2 * blk && ob < ib + blk)
            return fail(WL_EINVAL, "in overlaps the two parity blocks of out");
    }
    HopCall c1{};
    c1.gauge = gauge;
    c1.in[p] = in;
    c1.out[q] = tmp;
    c1.first_par = q;
    c1.npar = 1;
    c1.c = 1.0;
    c1.dag = dag;
    if (tw != 0.0) {   // tmp = A^-1 D in  (adjoint: A^-dag D^dag in)
        c1.c = 1.0 / (1.0 + tw * tw);
        c1.ta = dag ? tw : -tw;
    }
    hipError_t e = launch_hop(g, prec, flags & WL_LINK12, ph, c1, s);
    if (e == hipSuccess) {
        HopCall c2{};
        c2.gauge = gauge;
        c2.in[q] = tmp;
        c2.xs[p] = in;
        c2.out[p] = outp;
        c2.first_par = p;
        c2.npar = 1;
        c2.c = -kappa * kappa;
        c2.dag = dag;
        if (tw != 0.0) c2.tx = dag ? -tw : tw;   // A in - kappa^2 D tmp
        e = launch_hop(g, prec, flags & WL_LINK12, ph, c2, s);
    }
    return e == hipSuccess ? WL_OK : hip_fail(e, "wilson_dslash_eo");
}

// WL_CANON: the packed FP64 gauge field, b and x after the solver's own
// workspace, each on a 256-byte boundary
struct CanonStage {
    size_t gauge, b, x, end;
};
static CanonStage canon_stage(const Geom &g, uint32_t flags) {
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    CanonStage c;
    c.gauge = up(workspace_bytes(g, flags & ~WL_CANON));
    c.b = c.gauge + up(gauge_bytes(g, WL_F64, flags & WL_LINK12));
    c.x = c.b + up(2 * spinor_block_bytes(g, WL_F64));
    c.end = c.x + 2 * spinor_block_bytes(g, WL_F64);
    return c;
}

static size_t solve_workspace_bytes(const Geom &g, uint32_t flags) {
    return (flags & WL_CANON) ? canon_stage(g, flags).end : workspace_bytes(g, flags);
}

size_t wl_workspace_bytes(const int32_t dims[4], uint32_t flags, int32_t nrhs) {
    Geom g;
    std::string why;
    if (!make_geom(dims, &g, &why) || nrhs < 1 || nrhs > kMaxBatch) return 0;
    if (flags & WL_CANON) return nrhs == 1 ? canon_stage(g, flags).end : 0;
    return nrhs == 1 ? workspace_bytes(g, flags) : workspace_bytes_batch(g, flags, nrhs);
}

int wilson_dslash_batch(const void *gauge, const void *in, void *out, int32_t nrhs,
                        const int32_t dims[4], double kappa, const double phases[8],
                        uint32_t flags, void *stream) {
    Geom g;
    Phases ph;
    std::string why;
    int prec;
    if (!make_geom(dims, &g, &why) || !get_prec(flags, &prec, &why) ||
        !get_phases(phases, &ph, &why))
        return fail(WL_EINVAL, why);
    if (!gauge || !in || !out) return fail(WL_EINVAL, "NULL buffer");
    if (nrhs < 1 || nrhs > 65536) return fail(WL_EINVAL, "nrhs must be in 1..65536");
    const size_t blk = spinor_block_bytes(g, prec);
    const size_t fs = 2 * blk;
    const char *ib = static_cast<const char *>(in);
    const char *ob = static_cast<const char *>(out);
    if (ib < ob + fs * nrhs && ob < ib + fs * nrhs) return fail(WL_EINVAL, "in and out overlap");
    if (!std::isfinite(kappa)) return fail(WL_EINVAL, "kappa is not finite");
    if (flags & ~kKnownFlags) return fail(WL_EINVAL, "unknown flag bits");
    HopCall c{};
    c.gauge = gauge;
    c.in[0] = in;
    c.in[1] = ib + blk;
    c.out[0] = out;
    c.out[1] = static_cast<char *>(out) + blk;
    if (!(flags & WL_HOP)) {
        c.xs[0] = c.in[0];
        c.xs[1] = c.in[1];
        c.c = -kappa;
    } else {
        c.c = 1.0;
    }
    c.first_par = 0;
    c.npar = 2;
    c.dag = flags & WL_DAG;
    c.nrhs = nrhs;
    c.fstride = fs;
    const hipError_t e = launch_hop(g, prec, flags & WL_LINK12, ph, c,
                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wilson_dslash_batch");
}

size_t wl_problems_workspace_bytes(const wl_problem *p, int32_t n, uint32_t flags) {
    if (!p || n < 1) return 0;
    return problems_workspace_bytes(p, n, flags);
}

int solve_cg_problems(const wl_problem *p, int32_t n, const double phases[8], double tol,
                      int32_t maxiter, uint32_t flags, void *work, size_t work_bytes,
                      wl_solve_stats *stats, void *stream) {
    Phases ph;
    std::string why;
    if (!p || n < 1) return fail(WL_EINVAL, "no problems");
    if (!get_phases(phases, &ph, &why)) return fail(WL_EINVAL, why);
    if (flags & ~kKnownFlags) return fail(WL_EINVAL, "unknown flag bits");
    {
        const uint32_t inner = flags & WL_PREC_MASK;
        if (inner == WL_PREC_MASK || (inner != WL_F64 && !(flags & WL_MIXED)))
            return fail(WL_EINVAL, "solver buffers are FP64; a lower precision (WL_F32, WL_F16S) "
                                   "selects the inner solve of WL_MIXED");
        if (flags & (WL_DAG | WL_HOP))
            return fail(WL_EINVAL, "WL_DAG / WL_HOP do not apply to solves");
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(WL_EINVAL, "tol must be positive");
    if (maxiter < 1) return fail(WL_EINVAL, "maxiter must be >= 1");
    if (!work) return fail(WL_EINVAL, "NULL workspace");
    for (int i = 0; i < n; ++i) {
        Geom g;
        if (!make_geom(p[i].dims, &g, &why))
            return fail(WL_EINVAL, "problem " + std::to_string(i) + ": " + why);
        if (!p[i].gauge || !p[i].b || !p[i].x)
            return fail(WL_EINVAL, "problem " + std::to_string(i) + ": NULL buffer");
        if (p[i].b == p[i].x) return fail(WL_EINVAL, "problem " + std::to_string(i) + ": b == x");
        if (!std::isfinite(p[i].kappa))
            return fail(WL_EINVAL, "problem " + std::to_string(i) + ": kappa is not finite");
    }
    const size_t need = problems_workspace_bytes(p, n, flags);
    if (work_bytes < need)
        return fail(WL_EWORKSPACE, "workspace too small: need " + std::to_string(need) +
                                       " bytes, got " + std::to_string(work_bytes));
    const int st = run_problems(p, n, ph, tol, maxiter, flags, work,
                                static_cast<hipStream_t>(stream), stats, &why);
    if (st != WL_OK) g_last_error = why.empty() ? "at least one problem missed tol" : why;
    return st;
}

int solve_cg_batch(const void *gauge, const void *b, void *x, int32_t nrhs,
                   const int32_t dims[4], double kappa, const double phases[8], double tol,
                   int32_t maxiter, uint32_t flags, void *work, size_t work_bytes,
                   wl_solve_stats *stats, void *stream) {
    SolveIn in{};
    std::string why;
    if (!make_geom(dims, &in.g, &why) || !get_phases(phases, &in.ph, &why))
        return fail(WL_EINVAL, why);
    if (nrhs < 1 || nrhs > kMaxBatch)
        return fail(WL_EINVAL, "nrhs must be in 1.." + std::to_string(kMaxBatch));
    if (flags & ~kKnownFlags) return fail(WL_EINVAL, "unknown flag bits");
    {
        const uint32_t inner = flags & WL_PREC_MASK;
        if (inner == WL_PREC_MASK || (inner != WL_F64 && !(flags & WL_MIXED)))
            return fail(WL_EINVAL, "solver buffers are FP64; a lower precision (WL_F32, WL_F16S) "
                                   "selects the inner solve of WL_MIXED");
        if (flags & (WL_DAG | WL_HOP))
            return fail(WL_EINVAL, "WL_DAG / WL_HOP do not apply to solves");
    }
    if (!gauge || !b || !x || !work) return fail(WL_EINVAL, "NULL buffer");
    const size_t fs = 2 * spinor_block_bytes(in.g, WL_F64);
    const char *bb = static_cast<const char *>(b);
    const char *xb = static_cast<const char *>(x);
    if (bb < xb + fs * nrhs && xb < bb + fs * nrhs) return fail(WL_EINVAL, "b and x overlap");
    if (!std::isfinite(kappa)) return fail(WL_EINVAL, "kappa is not finite");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(WL_EINVAL, "tol must be positive");
    if (maxiter < 1) return fail(WL_EINVAL, "maxiter must be >= 1");
    const size_t need = workspace_bytes_batch(in.g, flags, nrhs);
    if (work_bytes < need)
        return fail(WL_EWORKSPACE, "workspace too small: need " + std::to_string(need) +
                                       " bytes, got " + std::to_string(work_bytes));
    in.gauge = gauge;
    in.b = b;
    in.x = x;
    in.kappa = kappa;
    in.tol = tol;
    in.maxiter = maxiter;
    in.flags = flags;
    in.work = work;
    in.s = static_cast<hipStream_t>(stream);
    const int st = run_cg_batch(in, nrhs, stats, &why);
    if (st != WL_OK) g_last_error = why.empty() ? "at least one right-hand side missed tol" : why;
    return st;
}

// Scratch of the allocation-free solve entry point: one array per GPU the
// library runs on, held until the process ends. Host code never uses the
// array's name as an address: scratch_address() looks up each device's copy
// once (with that device current) and the solver is handed that pointer.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void **out, std::string *why) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *why = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return WL_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *why = "device index out of range for the static scratch table";
        return WL_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return WL_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return WL_OK;
}
}  // namespace

static int solve_common(bool bicg, const void *gauge, const void *b, void *x,
                        const int32_t dims[4], double kappa, const double phases[8], double tol,
                        int32_t maxiter, uint32_t flags, void *work, size_t work_bytes,
                        wl_solve_stats *stats, void *stream, bool static_scratch = false,
                        double mu = 0.0) {
    SolveIn in{};
    if (!std::isfinite(mu)) return fail(WL_EINVAL, "mu is not finite");
    in.mu = mu;
    std::string why;
    if (!make_geom(dims, &in.g, &why) || !get_phases(phases, &in.ph, &why))
        return fail(WL_EINVAL, why);
    if (static_scratch) {
        if (flags & WL_CANON)
            return fail(WL_EINVAL, "solve_cg_noalloc takes packed fields (no WL_CANON)");
        if (flags & WL_GRAPH)
            return fail(WL_EINVAL, "solve_cg_noalloc: WL_GRAPH instantiates graphs, which "
                                   "allocates; use solve_cg for graph replay");
        const size_t need = workspace_bytes(in.g, flags);
        if (need > kStaticScratchBytes)
            return fail(WL_EWORKSPACE,
                        "solve_cg_noalloc: this solve needs " + std::to_string(need) +
                            " bytes of scratch, more than the static scratch of " +
                            std::to_string(kStaticScratchBytes) +
                            " bytes; use solve_cg with a workspace");
        const int e = scratch_address(&work, &why);
        if (e != WL_OK) return fail(e, why);
        work_bytes = kStaticScratchBytes;
        in.no_alloc = true;
    }
    if (flags & ~(kKnownFlags | WL_CANON)) return fail(WL_EINVAL, "unknown flag bits");
    const uint32_t inner = flags & WL_PREC_MASK;
    if (inner == WL_PREC_MASK || (inner != WL_F64 && !(flags & WL_MIXED)))
        return fail(WL_EINVAL, "solver buffers are FP64; a lower precision (WL_F32, WL_F16S) "
                               "selects the inner solve of WL_MIXED");
    if (flags & (WL_DAG | WL_HOP)) return fail(WL_EINVAL, "WL_DAG / WL_HOP do not apply to solves");
    if (!gauge || !b || !x || !work) return fail(WL_EINVAL, "NULL buffer");
    if (b == x) return fail(WL_EINVAL, "b and x alias");
    if (!std::isfinite(kappa)) return fail(WL_EINVAL, "kappa is not finite");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(WL_EINVAL, "tol must be positive");
    if (maxiter < 1) return fail(WL_EINVAL, "maxiter must be >= 1");
    const size_t need = solve_workspace_bytes(in.g, flags);
    if (work_bytes < need)
        return fail(WL_EWORKSPACE, "workspace too small: need " + std::to_string(need) +
                                       " bytes, got " + std::to_string(work_bytes));
    in.gauge = gauge;
    in.b = b;
    in.x = x;
    in.kappa = kappa;
    in.tol = tol;
    in.maxiter = maxiter;
    in.flags = flags & ~WL_CANON;
    in.work = work;
    in.s = static_cast<hipStream_t>(stream);
    const hipStream_t caller = in.s;
    if (flags & WL_CANON) {   // pack into the workspace's staging area
        const CanonStage c = canon_stage(in.g, flags);
        char *w = static_cast<char *>(work);
        hipError_t e = launch_pack_gauge(in.g, WL_F64, flags & WL_LINK12, gauge, w + c.gauge,
                                         caller);
        if (e == hipSuccess) e = launch_pack_spinor(in.g, WL_F64, b, w + c.b, caller);
        if (e == hipSuccess && (flags & WL_X0))
            e = launch_pack_spinor(in.g, WL_F64, x, w + c.x, caller);
        if (e != hipSuccess) return hip_fail(e, "packing the canonical fields");
        in.gauge = w + c.gauge;
        in.b = w + c.b;
        in.x = w + c.x;
    }
    int st;
    if (in.no_alloc) {
        const TuningSuspended no_tuning;   // tuning would create events
        st = run_solver(bicg, in, stats, &why);
    } else {
        st = run_solver(bicg, in, stats, &why);
    }
    if ((flags & WL_CANON) && st >= 0) {   // the solution (or best iterate) back
        hipError_t e = launch_unpack_spinor(in.g, WL_F64, in.x, x, caller);
        if (e == hipSuccess) e = hipStreamSynchronize(caller);
        if (e != hipSuccess) return hip_fail(e, "unpacking the solution");
    }
    if (st != WL_OK) {
        if (why.empty()) {
            static const char *names[] = {"ok", "not converged within maxiter",
                                          "breakdown (a Krylov scalar vanished or is not finite)",
                                          "stagnated"};
            why = st > 0 && st < 4 ? names[st] : "error";
        }
        g_last_error = why;
    }
    return st;
}

int solve_cg(const void *gauge, const void *b, void *x, const int32_t dims[4], double kappa,
             const double phases[8], double tol, int32_t maxiter, uint32_t flags, void *work,
             size_t work_bytes, wl_solve_stats *stats, void *stream) {
    return solve_common(false, gauge, b, x, dims, kappa, phases, tol, maxiter, flags, work,
                        work_bytes, stats, stream);
}

int solve_cg_tm(const void *gauge, const void *b, void *x, const int32_t dims[4], double kappa,
                double mu, const double phases[8], double tol, int32_t maxiter, uint32_t flags,
                void *work, size_t work_bytes, wl_solve_stats *stats, void *stream) {
    return solve_common(false, gauge, b, x, dims, kappa, phases, tol, maxiter, flags, work,
                        work_bytes, stats, stream, false, mu);
}

int solve_bicgstab_tm(const void *gauge, const void *b, void *x, const int32_t dims[4],
                      double kappa, double mu, const double phases[8], double tol,
                      int32_t maxiter, uint32_t flags, void *work, size_t work_bytes,
                      wl_solve_stats *stats, void *stream) {
    return solve_common(true, gauge, b, x, dims, kappa, phases, tol, maxiter, flags, work,
                        work_bytes, stats, stream, false, mu);
}

int solve_cg_noalloc(const void *gauge, const void *b, void *x, const int32_t dims[4],
                     double kappa, const double phases[8], double tol, int32_t maxiter,
                     uint32_t flags, wl_solve_stats *stats, void *stream) {
    return solve_common(false, gauge, b, x, dims, kappa, phases, tol, maxiter, flags, nullptr, 0,
                        stats, stream, true);
}

int solve_bicgstab(const void *gauge, const void *b, void *x, const int32_t dims[4],
                   double kappa, const double phases[8], double tol, int32_t maxiter,
                   uint32_t flags, void *work, size_t work_bytes, wl_solve_stats *stats,
                   void *stream) {
    return solve_common(true, gauge, b, x, dims, kappa, phases, tol, maxiter, flags, work,
                        work_bytes, stats, stream);
}

size_t wl_meson_workspace_bytes(const int32_t dims[4]) {
    Geom g;
    std::string why;
    if (!make_geom(dims, &g, &why)) return 0;
    return meson_workspace_bytes(g);
}

int wl_meson_correlators(const void *props, const int32_t dims[4], int32_t t0, double *corr,
                         void *work, size_t work_bytes, void *stream) {
    Geom g;
    std::string why;
    if (!make_geom(dims, &g, &why)) return fail(WL_EINVAL, why);
    if (!props || !corr || !work) return fail(WL_EINVAL, "NULL buffer");
    if (t0 < 0 || t0 >= dims[3]) return fail(WL_EINVAL, "t0 must be a time slice of the lattice");
    const size_t need = meson_workspace_bytes(g);
    if (work_bytes < need)
        return fail(WL_EWORKSPACE, "workspace too small: need " + std::to_string(need) +
                                       " bytes, got " + std::to_string(work_bytes));
    const hipError_t e = launch_meson(g, props, t0, corr, work, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_meson_correlators");
}

static int heatbath_common(void *gauge, bool packed, const int32_t dims[4], double beta,
                           int32_t nsweeps, uint32_t sweep0, uint32_t seed, void *stream) {
    Geom g;
    std::string why;
    if (!make_geom(dims, &g, &why)) return fail(WL_EINVAL, why);
    if (!gauge) return fail(WL_EINVAL, "NULL buffer");
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(WL_EINVAL, "beta must be positive");
    if (nsweeps < 0) return fail(WL_EINVAL, "nsweeps must be >= 0");
    const hipError_t e = launch_heatbath_field(g, gauge, packed, beta, nsweeps, sweep0, seed,
                                               static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, packed ? "wl_heatbath_packed" : "wl_heatbath");
}

int wl_heatbath(void *gauge, const int32_t dims[4], double beta, int32_t nsweeps,
                uint32_t sweep0, uint32_t seed, void *stream) {
    return heatbath_common(gauge, false, dims, beta, nsweeps, sweep0, seed, stream);
}

int wl_heatbath_packed(void *gauge, const int32_t dims[4], double beta, int32_t nsweeps,
                       uint32_t sweep0, uint32_t seed, void *stream) {
    return heatbath_common(gauge, true, dims, beta, nsweeps, sweep0, seed, stream);
}

size_t wl_plaquette_workspace_bytes(const int32_t dims[4]) {
    Geom g;
    std::string why;
    if (!make_geom(dims, &g, &why)) return 0;
    return plaquette_workspace_bytes(g);
}

static int plaquette_common(const void *gauge, bool packed, const int32_t dims[4],
                            double *out, void *work, size_t work_bytes, void *stream) {
    Geom g;
    std::string why;
    if (!make_geom(dims, &g, &why)) return fail(WL_EINVAL, why);
    if (!gauge || !out || !work) return fail(WL_EINVAL, "NULL buffer");
    const size_t need = plaquette_workspace_bytes(g);
    if (work_bytes < need)
        return fail(WL_EWORKSPACE, "workspace too small: need " + std::to_string(need) +
                                       " bytes, got " + std::to_string(work_bytes));
    const hipError_t e = launch_plaquette_field(g, gauge, packed, out, work,
                                                static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, packed ? "wl_plaquette_packed" : "wl_plaquette");
}

int wl_plaquette(const void *gauge, const int32_t dims[4], double *out, void *work,
                 size_t work_bytes, void *stream) {
    return plaquette_common(gauge, false, dims, out, work, work_bytes, stream);
}

int wl_plaquette_packed(const void *gauge, const int32_t dims[4], double *out, void *work,
                        size_t work_bytes, void *stream) {
    return plaquette_common(gauge, true, dims, out, work, work_bytes, stream);
}

int wl_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst) return fail(WL_EINVAL, "NULL buffer");
    const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
    if ((a | b | bytes) & 15) return fail(WL_EINVAL, "pointers and size must be multiples of 16");
    if (a < b + bytes && b < a + bytes) return fail(WL_EINVAL, "src and dst overlap");
    const hipError_t e = launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_stream_copy");
}

size_t wl_tuning_report(char *buf, size_t len) {
    const std::string r = tuning_report();
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, r.size());
        std::memcpy(buf, r.data(), n);
        buf[n] = '\0';
    }
    return r.size();
}

int wl_server_create(const wl_server_config *cfg, wl_server **out) {
    std::string why;
    Phases ph;
    if (!cfg || !out) return fail(WL_EINVAL, "NULL config or output");
    *out = nullptr;
    if (cfg->hbm_budget == 0) return fail(WL_EINVAL, "hbm_budget must be positive");
    if (cfg->slots < 1 || cfg->slots > 64) return fail(WL_EINVAL, "slots must be in 1..64");
    if (cfg->merge < 0 || cfg->merge > kMaxBatch) return fail(WL_EINVAL, "merge must be in 0..64");
    if (!get_phases(cfg->phases, &ph, &why)) return fail(WL_EINVAL, why);
    if (!(cfg->site_slack >= 0.0) || !std::isfinite(cfg->site_slack))
        return fail(WL_EINVAL, "site_slack must be finite and >= 0");
    const uint32_t flags = cfg->flags;
    if (flags & WL_CANON) return fail(WL_EINVAL, "the server takes packed fields (no WL_CANON)");
    if (flags & ~kKnownFlags) return fail(WL_EINVAL, "unknown flag bits");
    const uint32_t inner = flags & WL_PREC_MASK;
    if (inner == WL_PREC_MASK || (inner != WL_F64 && !(flags & WL_MIXED)))
        return fail(WL_EINVAL, "a lower precision (WL_F32, WL_F16S) selects the inner solve of "
                               "WL_MIXED");
    if (flags & (WL_DAG | WL_HOP)) return fail(WL_EINVAL, "WL_DAG / WL_HOP do not apply to solves");
    if (!(cfg->tol > 0.0) || !std::isfinite(cfg->tol)) return fail(WL_EINVAL, "tol must be positive");
    if (cfg->maxiter < 1) return fail(WL_EINVAL, "maxiter must be >= 1");
    const int st = server_create(*cfg, ph, out, &why);
    return st == WL_OK ? WL_OK : fail(st, why);
}

int wl_server_submit(wl_server *srv, const wl_problem *p, uint64_t *ticket) {
    std::string why;
    Geom g;
    if (!srv || !p || !ticket) return fail(WL_EINVAL, "NULL server, problem or ticket");
    if (!make_geom(p->dims, &g, &why)) return fail(WL_EINVAL, why);
    if (!p->gauge || !p->b || !p->x) return fail(WL_EINVAL, "NULL buffer");
    if (p->b == p->x) return fail(WL_EINVAL, "b and x alias");
    if (!std::isfinite(p->kappa)) return fail(WL_EINVAL, "kappa is not finite");
    const int st = server_submit(srv, *p, g, ticket, &why);
    return st == WL_OK ? WL_OK : fail(st, why);
}

static int server_status(int st, const std::string &why) {
    if (st == WL_OK) return WL_OK;
    if (st < 0) return fail(st, why);
    static const char *names[] = {"ok", "not converged within maxiter",
                                  "breakdown (a Krylov scalar vanished or is not finite)",
                                  "stagnated"};
    g_last_error = st > 0 && st < 4 ? names[st] : "error";
    return st;
}

int wl_server_wait(wl_server *srv, uint64_t ticket, wl_solve_stats *stats,
                   wl_request_times *times) {
    std::string why;
    if (!srv) return fail(WL_EINVAL, "NULL server");
    return server_status(server_wait(srv, ticket, stats, times, &why), why);
}

int wl_server_next(wl_server *srv, uint64_t *ticket, wl_solve_stats *stats,
                   wl_request_times *times) {
    std::string why;
    if (!srv || !ticket) return fail(WL_EINVAL, "NULL server or ticket");
    return server_status(server_next(srv, ticket, stats, times, &why), why);
}

int32_t wl_server_pending(wl_server *srv) { return srv ? server_pending(srv) : 0; }

int wl_server_destroy(wl_server *srv) {
    if (!srv) return WL_OK;
    const int st = server_destroy(srv);
    return st == WL_OK ? WL_OK : fail(st, "HIP error releasing the server");
}

}  // extern "C"
