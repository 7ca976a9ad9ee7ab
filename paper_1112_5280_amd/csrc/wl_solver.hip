// wl_solver.hip -- Krylov solvers for M x = b (paper Sec. 4: the inversion of
// the fermion matrix for point-source propagators; Sec. 3: even-odd
// preconditioning).
//
//   CGNR      Hestenes-Stiefel CG on M^dag M x = M^dag b.
//   BiCGStab  van der Vorst's BiCGStab on M.
//   WL_EO     both run on the Schur system Mhat_e x_e = b_e + kappa D_eo b_o,
//             Mhat_e = 1 - kappa^2 D_eo D_oe, then x_o = b_o + kappa D_oe x_e.
//   WL_MIXED  Krylov iterations in FP32 or FP16 storage. CG keeps one Krylov
//             sequence with reliable updates: whenever the low-precision
//             residual has dropped by delta, x += x_lo in FP64 and the residual
//             is recomputed in FP64 and copied back. BiCGStab uses FP64 defect
//             correction: an inner solve of M e = r, then x += e.
//
// Every solve finishes with the FP64 true residual ||b - M x|| / ||b|| on the
// full lattice; when it misses tol the Krylov loop restarts from x with a
// tighter inner target. The Krylov loops keep all scalars on the device; the
// host enqueues a chunk of iterations and then reads one small status block.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <deque>
#include <initializer_list>
#include <map>
#include <thread>
#include <vector>

#include "wl_host.h"

namespace wl {

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
constexpr int kVec64 = 9;   // FP64 full spinors (the last keeps the best iterate)
constexpr int kVecBatch = 8;   // FP64 full spinors per RHS of a batched solve
constexpr int kVec32 = 10;  // FP32 full spinors (mixed precision)
constexpr size_t kAlign = 256;

static size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// storage precision of the inner (low-precision) Krylov vectors of WL_MIXED
static int lo_prec(uint32_t flags) {
    return (flags & WL_PREC_MASK) == WL_F16S ? WL_F16S : WL_F32;
}

struct Workspace {
    Scalars *sc;
    double *partials;
    char *v64[kVec64];
    void *gauge32;
    char *v32[kVec32];
};

static size_t header_bytes(const Geom &g) {
    return align_up(4096 + sizeof(double) * kMaxSums * 2 * size_t(g.bpp));
}

size_t workspace_bytes(const Geom &g, uint32_t flags) {
    size_t n = header_bytes(g) + kVec64 * align_up(2 * spinor_block_bytes(g, WL_F64));
    if (flags & WL_MIXED)
        n += align_up(gauge_bytes(g, lo_prec(flags), flags & WL_LINK12)) +
             kVec32 * align_up(2 * spinor_block_bytes(g, lo_prec(flags)));
    return n;
}

static Workspace carve(const Geom &g, uint32_t flags, void *work) {
    Workspace ws{};
    char *p = static_cast<char *>(work);
    ws.sc = reinterpret_cast<Scalars *>(p);
    ws.partials = reinterpret_cast<double *>(p + 4096);
    p += header_bytes(g);
    const size_t f64 = align_up(2 * spinor_block_bytes(g, WL_F64));
    for (int k = 0; k < kVec64; ++k, p += f64) ws.v64[k] = p;
    if (flags & WL_MIXED) {
        ws.gauge32 = p;
        p += align_up(gauge_bytes(g, lo_prec(flags), flags & WL_LINK12));
        const size_t f32 = align_up(2 * spinor_block_bytes(g, lo_prec(flags)));
        for (int k = 0; k < kVec32; ++k, p += f32) ws.v32[k] = p;
    }
    return ws;
}

// ---------------------------------------------------------------------------
// Host-side status readback
// ---------------------------------------------------------------------------
struct Fail {
    hipError_t err;
};

static void check(hipError_t e) {
    if (e != hipSuccess) throw Fail{e};
}

// Per-thread pinned host buffer for status readbacks (kMaxBatch scalar
// blocks), released when the thread ends.
struct PinnedScalars {
    Scalars *p = nullptr;
    ~PinnedScalars() {
        if (p) (void)hipHostFree(p);
    }
};

// A solve that may allocate nothing reads its status through plain host
// memory instead (pageable copies are slower, but need no allocation).
thread_local bool t_pageable_status = false;

struct PageableStatus {
    bool prev;
    explicit PageableStatus(bool on) : prev(t_pageable_status) { t_pageable_status = prev || on; }
    ~PageableStatus() { t_pageable_status = prev; }
};

static Scalars *host_scalars() {
    if (t_pageable_status) {
        thread_local Scalars plain[kMaxBatch];
        return plain;
    }
    thread_local PinnedScalars buf;
    if (!buf.p)
        check(hipHostMalloc(reinterpret_cast<void **>(&buf.p), sizeof(Scalars) * kMaxBatch,
                            hipHostMallocDefault));
    return buf.p;
}

static Scalars read_scalars(const Scalars *dev, hipStream_t s) {
    Scalars *h = host_scalars();
    check(hipMemcpyAsync(h, dev, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    return *h;
}

// ---------------------------------------------------------------------------
// The operator of a Krylov solve, in one storage precision
// ---------------------------------------------------------------------------
struct Space {
    const Geom *g;
    int prec;
    bool link12;
    Phases ph;
    const void *gauge;
    double kappa;
    bool eo;
    hipStream_t s;
    Scalars *sc;
    double *partials;
    void *tmp;               // one parity block for the eo intermediate
    // model cost bookkeeping
    double applies = 0;      // applications of A or A^dag
    // batches: nrhs fields per vector, fstride bytes apart; scalars sc[0..nrhs)
    int nrhs = 1;
    size_t fstride = 0;
    bool graph = false;      // replay chunks of Krylov iterations from a HIP graph
    // independent problems: per-RHS gauge fields (device table) and kappa
    // (sc[r].kappa); the hop coefficient is then cmul * kappa_r^cpow
    const void *const *gtab = nullptr;
    bool per_kappa = false;
    // twisted mass: tw = 2 kappa mu (0: Wilson). The operator is then
    // M = A - kappa D_W with A = 1 + i tw g5; its even-odd form is the Schur
    // complement S = A - kappa^2 D_eo A^-1 D_oe, A^-1 = (1 - i tw g5)/(1 + tw^2),
    // and the adjoints take -tw (A^dag = 1 - i tw g5, g5 D g5 = D^dag).
    double tw = 0.0;

    // hop coefficient c = cmul * kappa^cpow, for the shared or per-RHS kappa
    void coef(HopCall &c, double cmul, int cpow) const {
        c.gtab = gtab;
        if (per_kappa) {
            c.ksc = sc;
            c.cmul = cmul;
            c.cpow = cpow;
        } else {
            c.c = cmul * (cpow == 2 ? kappa * kappa : cpow == 1 ? kappa : 1.0);
        }
    }

    int npar() const { return eo ? 1 : 2; }
    size_t blk() const { return spinor_block_bytes(*g, prec); }
    void *par(void *full, int q) const { return static_cast<char *>(full) + q * blk(); }
    const void *par(const void *full, int q) const {
        return static_cast<const char *>(full) + q * blk();
    }

    Reduce red(int epi) const { return Reduce{partials, sc->sums, epi, sc}; }

    // out = A in, A = M (full) or Mhat_e (eo), or the adjoint; optional fused
    // reduction (norm of out / <aux, out> / <out, in> and ||out||^2).
    void apply(const void *in, void *out, bool dag, int epi, const void *aux, const int *skip) {
        const Reduce r = red(epi);
        const Reduce *rp = epi == kEpiNone ? nullptr : &r;
        if (!eo) {
            HopCall c{};
            c.gauge = gauge;
            c.in[0] = in; c.in[1] = par(in, 1);
            c.xs[0] = in; c.xs[1] = par(in, 1);
            c.aux[0] = aux; c.aux[1] = aux ? par(aux, 1) : nullptr;
            c.out[0] = out; c.out[1] = par(out, 1);
            c.first_par = 0; c.npar = 2; c.dag = dag; c.skip = skip; c.red = rp;
            c.nrhs = nrhs; c.fstride = fstride;
            coef(c, -1.0, 1);
            if (tw != 0.0) c.tx = dag ? -tw : tw;
            check(launch_hop(*g, prec, link12, ph, c, s));
        } else {
            HopCall c1{};
            c1.gauge = gauge;
            c1.in[0] = in;
            c1.out[1] = tmp;
            c1.first_par = 1; c1.npar = 1; c1.dag = dag; c1.skip = skip;
            c1.nrhs = nrhs; c1.fstride = fstride;
            coef(c1, 1.0, 0);
            if (tw != 0.0) {   // tmp = A^-1 D in  (adjoint: A^-dag D^dag in)
                c1.c = 1.0 / (1.0 + tw * tw);
                c1.ta = dag ? tw : -tw;
            }
            check(launch_hop(*g, prec, link12, ph, c1, s));
            HopCall c2{};
            c2.gauge = gauge;
            c2.in[1] = tmp;
            c2.xs[0] = in;
            c2.aux[0] = aux;
            c2.out[0] = out;
            c2.first_par = 0; c2.npar = 1; c2.dag = dag; c2.skip = skip;
            c2.red = rp;
            c2.nrhs = nrhs; c2.fstride = fstride;
            coef(c2, -1.0, 2);
            if (tw != 0.0) c2.tx = dag ? -tw : tw;   // A in - kappa^2 D tmp
            check(launch_hop(*g, prec, link12, ph, c2, s));
        }
        applies += 1;
    }

    // The CG step after t = A p: q = A^dag t, x += alpha p, r -= alpha q and
    // ||r||^2 (kEpiCgRr). On the even-odd system the update runs in the
    // epilogue of the adjoint's last hop (one RHS per thread, which is also
    // the tuned shape of batched even-odd hops) and q is never stored: 192 B
    // per FP32 site and iteration less. The full-lattice system keeps the hop
    // and the update pass; in FP64 and FP32 both forms give the same bits.
    static bool fuses_cg(bool eo) { return eo; }
    void cg_step(const void *t, void *q, void *x, void *p, void *r, const int *skip) {
        if (!fuses_cg(eo)) {
            apply(t, q, true, kEpiNone, nullptr, skip);
            blas(kOpCgXR, x, p, r, q, nullptr, nullptr, kEpiCgRr);
            return;
        }
        HopCall c1{};
        c1.gauge = gauge;
        c1.in[0] = t;
        c1.out[1] = tmp;
        c1.first_par = 1; c1.npar = 1; c1.dag = true; c1.skip = skip;
        c1.nrhs = nrhs; c1.fstride = fstride;
        coef(c1, 1.0, 0);
        if (tw != 0.0) {   // tmp = A^-dag D^dag t
            c1.c = 1.0 / (1.0 + tw * tw);
            c1.ta = tw;
        }
        check(launch_hop(*g, prec, link12, ph, c1, s));
        const Reduce rr = red(kEpiCgRr);
        HopCall c2{};
        c2.gauge = gauge;
        c2.in[1] = tmp;
        c2.xs[0] = t;
        c2.out[0] = q;
        c2.first_par = 0; c2.npar = 1; c2.dag = true; c2.skip = skip;
        c2.red = &rr;
        c2.nrhs = nrhs; c2.fstride = fstride;
        coef(c2, -1.0, 2);
        if (tw != 0.0) c2.tx = -tw;
        c2.cg[0] = x; c2.cg[1] = p; c2.cg[2] = r;
        check(launch_hop(*g, prec, link12, ph, c2, s));
        applies += 1;
    }

    void blas(int op, void *v0, void *v1 = nullptr, void *v2 = nullptr, void *v3 = nullptr,
              void *v4 = nullptr, void *v5 = nullptr, int epi = kEpiNone, bool use_skip = true,
              double a = 0.0, double b = 0.0) {
        const Reduce r = red(epi);
        BlasCall c{};
        c.op = op;
        c.npar = npar();
        c.v[0] = v0; c.v[1] = v1; c.v[2] = v2; c.v[3] = v3; c.v[4] = v4; c.v[5] = v5;
        c.a = a;
        c.b = b;
        c.sc = sc;
        c.skip = use_skip ? &sc->done : nullptr;
        c.red = (op == kOpNorm2 || op == kOpXmy || op == kOpCgXR || op == kOpBiXR ||
                 op == kOpCopyNorm2 || op == kOpCopy2Norm2 || op == kOpNormDot) ? &r : nullptr;
        c.nrhs = nrhs;
        c.fstride = fstride;
        check(launch_blas(*g, prec, c, s));
    }

    // sum0 of the last reduction, read back to the host
    double norm2(const void *v) {
        blas(kOpNorm2, const_cast<void *>(v), nullptr, nullptr, nullptr, nullptr, nullptr,
             kEpiNone, false);
        return read_scalars(sc, s).sums[0];
    }
};

// Iterations per host check: small enough to stop soon after convergence,
// large enough to hide the readback.
static int chunk_for(const Geom &g) { return g.Vh >= (1 << 18) ? 4 : 16; }

// Iterations still needed to bring ||r||^2 from h.rr down to h.target at the
// rate of the last `done` iterations (which started from rr_before); -1 when
// there is no estimate (no progress measured, or the target already met).
static double cg_need(double rr_before, int done, const Scalars &h) {
    if (done <= 0 || !(h.target > 0.0) || !(h.rr > h.target) || !(rr_before > h.rr)) return -1.0;
    return std::log(h.target / h.rr) / (std::log(h.rr / rr_before) / done);
}

// Length of the next chunk of CG iterations: the estimate above plus one,
// rounded up to a multiple of 4 (few distinct graph lengths), at most the
// lattice's chunk. CG does not converge at a fixed rate, so a short estimate
// costs one more chunk and a long one runs iterations the device skips once
// the target is met; the arithmetic is the same either way, and on small
// lattices, where every launch costs more than its work, the trailing
// skipped launches of a full chunk are saved.
static int next_chunk(int cmax, double need) {
    if (!(need >= 0.0) || !(need < cmax)) return cmax;
    const int n = int(std::ceil(need)) + 1;
    return std::min(cmax, (n + 3) / 4 * 4);
}

// ---------------------------------------------------------------------------
// Chunks of Krylov iterations, enqueued directly or -- with WL_GRAPH --
// captured into a HIP graph and replayed. A chunk holds kernel launches only
// (no memset, no host work); the host reads the status block between chunks.
// Instantiated graphs are cached per host thread under a key of everything
// their kernel arguments depend on (the loop kind, chunk length, stream,
// operator, buffers and scalar block), so a later solve with the same
// buffers replays them without capturing again.
// ---------------------------------------------------------------------------
using GraphKey = std::vector<uint64_t>;

struct GraphCache {
    static constexpr size_t kMax = 64;
    std::map<GraphKey, hipGraphExec_t> execs;
    std::deque<GraphKey> order;   // insertion order, for eviction
    ~GraphCache() {
        for (auto &kv : execs) (void)hipGraphExecDestroy(kv.second);
    }
    hipGraphExec_t find(const GraphKey &k) const {
        auto it = execs.find(k);
        return it == execs.end() ? nullptr : it->second;
    }
    void put(const GraphKey &k, hipGraphExec_t e) {
        if (execs.size() >= kMax) {
            auto it = execs.find(order.front());
            if (it != execs.end()) {
                (void)hipGraphExecDestroy(it->second);
                execs.erase(it);
            }
            order.pop_front();
        }
        execs[k] = e;
        order.push_back(k);
    }
};

static GraphCache &graph_cache() {
    thread_local GraphCache c;
    return c;
}

static uint64_t bits_of(double v) {
    uint64_t u;
    std::memcpy(&u, &v, sizeof u);
    return u;
}

// The key of a chunk loop of kind `tag` on space k over the given vectors
static GraphKey chunk_key(int tag, const Space &k, std::initializer_list<const void *> vecs) {
    GraphKey key{uint64_t(tag), uint64_t(reinterpret_cast<uintptr_t>(k.s)), uint64_t(k.prec),
                 uint64_t(k.link12), uint64_t(k.eo), uint64_t(k.nrhs), uint64_t(k.fstride),
                 uint64_t(reinterpret_cast<uintptr_t>(k.gauge)),
                 uint64_t(reinterpret_cast<uintptr_t>(k.gtab)), uint64_t(k.per_kappa),
                 bits_of(k.kappa), bits_of(k.tw),
                 uint64_t(reinterpret_cast<uintptr_t>(k.sc)),
                 uint64_t(reinterpret_cast<uintptr_t>(k.partials)),
                 uint64_t(reinterpret_cast<uintptr_t>(k.tmp))};
    for (int mu = 0; mu < 4; ++mu) {
        key.push_back(uint64_t(k.g->L[mu]));
        key.push_back(bits_of(k.ph.re[mu]));
        key.push_back(bits_of(k.ph.im[mu]));
    }
    for (const void *v : vecs) key.push_back(uint64_t(reinterpret_cast<uintptr_t>(v)));
    return key;
}

struct ChunkRunner {
    hipStream_t s;
    bool graph;
    GraphKey key;

    ChunkRunner(hipStream_t s_, bool graph_, GraphKey key_ = {})
        : s(s_), graph(graph_), key(std::move(key_)) {}
    ChunkRunner(const ChunkRunner &) = delete;
    ChunkRunner &operator=(const ChunkRunner &) = delete;

    template <class F>
    void run(int n, F &&enqueue) {
        if (!graph) {
            enqueue(n);
            return;
        }
        GraphKey k = key;
        k.push_back(uint64_t(n));
        GraphCache &cache = graph_cache();
        hipGraphExec_t exec = cache.find(k);
        if (!exec) {
            check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipGraph_t gr = nullptr;
            try {
                enqueue(n);
            } catch (...) {
                (void)hipStreamEndCapture(s, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                throw;
            }
            check(hipStreamEndCapture(s, &gr));
            const hipError_t e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            check(e);
            cache.put(k, exec);
        }
        check(hipGraphLaunch(exec, s));
    }
};

// The library's own stream for captured solves (graphs cannot be captured on
// the null stream); default priority, one per host thread.
struct OwnedStream {
    hipStream_t s = nullptr;
    ~OwnedStream() {
        if (s) (void)hipStreamDestroy(s);
    }
};

static hipStream_t graph_stream() {
    thread_local OwnedStream os;
    if (!os.s) check(hipStreamCreateWithFlags(&os.s, hipStreamNonBlocking));
    return os.s;
}

constexpr int kStallWindow = 2000;

// ---------------------------------------------------------------------------
// CGNR core: iterate on A^dag A x = A^dag rhs until ||r||^2 <= target
// ---------------------------------------------------------------------------
struct CoreResult {
    int iters;
    int status;   // WL_OK (target met), WL_NOCONV, WL_BREAKDOWN, WL_STAGNATED
    double rr;
    int updates = 0;   // reliable updates (mixed CG)
};

static CoreResult cg_core(Space &k, const void *rhs, void *x, void *r, void *p, void *t, void *q,
                          double target, int maxit) {
    // r = A^dag (rhs - A x);  p = r
    check(launch_set_target(k.sc, target, k.s));
    k.apply(x, t, false, kEpiNone, nullptr, nullptr);
    k.blas(kOpXmy, const_cast<void *>(rhs), t, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
    k.apply(t, r, true, kEpiNone, nullptr, nullptr);
    k.blas(kOpCopyNorm2, r, p, nullptr, nullptr, nullptr, nullptr, kEpiCgInit, false);
    const int chunk = chunk_for(*k.g);
    int done_it = 0;
    Scalars h = read_scalars(k.sc, k.s);
    ChunkRunner runner(k.s, k.graph, chunk_key(1, k, {x, r, p, t, q}));
    int len = chunk;
    while (!h.done && done_it < maxit) {
        const int n = std::min(len, maxit - done_it);
        const double rr0 = h.rr;
        const int it0 = h.iter;
        runner.run(n, [&](int m) {
            for (int it = 0; it < m; ++it) {
                const int *skip = &k.sc->done;
                k.apply(p, t, false, kEpiCgPap, nullptr, skip);    // t = A p, pap = |t|^2
                k.cg_step(t, q, x, p, r, skip);                    // q = A^dag t; x, r, rr
                k.blas(kOpCgP, r, p);
            }
        });
        h = read_scalars(k.sc, k.s);
        done_it = h.iter;
        len = next_chunk(chunk, cg_need(rr0, h.iter - it0, h));
    }
    CoreResult res;
    res.iters = h.iter;
    res.rr = h.rr;
    res.status = h.done ? h.status : WL_NOCONV;
    return res;
}

// ---------------------------------------------------------------------------
// Mixed-precision CGNR with reliable updates. CG iterates in the FP32 space
// k32 on (r, p, x_lo); once ||r||^2 has dropped by delta^2 since the last
// update (the device loop stops itself there), the FP32 correction x_lo is
// added to the FP64 solution x, the normal-equations residual
// A^dag (rhs - A x) is recomputed in FP64 and copied back into r, and the
// iteration continues along the same search direction p.
// ---------------------------------------------------------------------------
struct LoVecs {
    void *r, *p, *t, *q, *x;
};

// residual reduction between reliable updates, per inner precision
// (measured on the 32^3 x 64 solve: FP32 inner 0.1 -> 11 updates, 147 ms;
// 3e-3 -> 5 updates; 1e-4 -> 4 updates, 1-2 % faster than 3e-3 with the same
// 152 iterations, and the same iterations on 16^3 x 32, 8^4 and the 12
// point sources of 24^3 x 48. FP16 inner 0.2 -> 15 updates, 99 ms; 0.1 -> 11,
// 93 ms but smaller lattices then stall below the FP16 noise floor; 0.05 adds
// iterations; 0.02 needs 255.) WL_DELTA_F32 / WL_DELTA_F16 override them.
static double reliable_delta(int prec) {
    const char *v = std::getenv(prec == WL_F16S ? "WL_DELTA_F16" : "WL_DELTA_F32");
    const double d = v ? std::atof(v) : 0.0;
    if (d > 0.0 && d < 1.0) return d;
    return prec == WL_F16S ? 0.2 : 1e-4;
}

// An inner loop whose residual has not halved within this many iterations has
// reached the noise floor of its precision: update from FP64 now.
constexpr int kInnerStall = 300;

static CoreResult cg_reliable(Space &k64, Space &k32, const void *rhs, void *x, void *r64,
                              void *t64, const LoVecs &lo, double target, double delta,
                              int maxit) {
    const int npar = k64.npar();
    const int chunk = chunk_for(*k64.g);
    auto residual64 = [&]() {
        k64.apply(x, t64, false, kEpiNone, nullptr, nullptr);
        k64.blas(kOpXmy, const_cast<void *>(rhs), t64, nullptr, nullptr, nullptr, nullptr,
                 kEpiNone, false);
        k64.apply(t64, r64, true, kEpiNone, nullptr, nullptr);
        return k64.norm2(r64);
    };
    // load the FP64 residual into r, clear x_lo, and set the device stop point
    auto reload = [&](double rr) {
        check(launch_convert_spinor(*k64.g, npar, WL_F64, r64, k32.prec, lo.r, k64.s));
        k32.blas(kOpZero, lo.x, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
        check(launch_set_target(k32.sc, std::max(target, delta * delta * rr), k32.s));
    };
    CoreResult res{0, WL_NOCONV, 0.0, 0};
    double rr = residual64();
    res.rr = rr;
    if (!std::isfinite(rr)) {
        res.status = WL_BREAKDOWN;
        return res;
    }
    if (rr <= target) {
        res.status = WL_OK;
        return res;
    }
    reload(rr);
    k32.blas(kOpCopyNorm2, lo.r, lo.p, nullptr, nullptr, nullptr, nullptr, kEpiCgInit, false);
    int its = 0, stale = 0;
    ChunkRunner runner(k32.s, k32.graph, chunk_key(2, k32, {lo.p, lo.t, lo.q, lo.x, lo.r}));
    while (its < maxit) {
        Scalars h = read_scalars(k32.sc, k32.s);
        double best = h.rr;
        int best_it = h.iter;
        int len = chunk;
        while (!h.done && its + h.iter < maxit) {
            const int n = std::min(len, maxit - its - h.iter);
            const double rr0 = h.rr;
            const int it0 = h.iter;
            runner.run(n, [&](int m) {
                for (int it = 0; it < m; ++it) {
                    const int *skip = &k32.sc->done;
                    k32.apply(lo.p, lo.t, false, kEpiCgPap, nullptr, skip);
                    k32.cg_step(lo.t, lo.q, lo.x, lo.p, lo.r, skip);
                    k32.blas(kOpCgP, lo.r, lo.p);
                }
            });
            h = read_scalars(k32.sc, k32.s);
            len = next_chunk(chunk, cg_need(rr0, h.iter - it0, h));
            if (h.rr < 0.5 * best) {
                best = h.rr;
                best_it = h.iter;
            } else if (h.iter - best_it > kInnerStall) {
                break;   // at the inner precision's noise floor: reliable update now
            }
        }
        its += h.iter;
        // reliable update: x += x_lo in FP64, fresh FP64 residual
        check(launch_accum_lo(*k64.g, npar, k32.prec, lo.x, x, k64.s));
        const double rr_new = residual64();
        res.updates += 1;
        res.rr = rr_new;
        if (!std::isfinite(rr_new)) {
            res.status = WL_BREAKDOWN;
            break;
        }
        if (rr_new <= target) {
            res.status = WL_OK;
            break;
        }
        stale = rr_new < 0.5 * rr ? 0 : stale + 1;
        if (stale > 8) {
            res.status = WL_STAGNATED;
            break;
        }
        rr = rr_new;
        reload(rr);
        // sc->rr = ||r||^2 of the reloaded residual
        k32.blas(kOpNorm2, lo.r, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiCgInit, false);
        // The device loop stopped right after the x, r update, so the direction
        // update of that iteration was skipped: apply it now with the reloaded
        // residual, beta = ||r||^2 / ||r_old||^2 (||r_old||^2 = rr / beta).
        if (h.done && h.status == WL_OK && h.beta > 0.0 && h.rr > 0.0) {
            check(launch_beta_ratio(k32.sc, h.rr / h.beta, k32.s));
            k32.blas(kOpCgP, lo.r, lo.p, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
        } else {   // broken down or out of iterations: restart the direction from r
            k32.blas(kOpCopy, lo.r, lo.p, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
        }
    }
    res.iters = its;
    return res;
}

// ---------------------------------------------------------------------------
// BiCGStab core: iterate on A x = rhs until ||r||^2 <= target
// ---------------------------------------------------------------------------
// The shadow vector of a fresh BiCGStab sequence: rhat = r, or (after a
// breakdown) a pseudo-random field of the given nonzero seed.
static void bicg_shadow(Space &k, void *r, void *rh, uint64_t seed) {
    if (!seed) {
        k.blas(kOpCopyNorm2, r, rh, nullptr, nullptr, nullptr, nullptr, kEpiBiInit, false);
        return;
    }
    k.blas(kOpRandom, rh, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false,
           double(seed));
    k.blas(kOpNormDot, rh, r, nullptr, nullptr, nullptr, nullptr, kEpiBiInitShadow, false);
}

static CoreResult bicg_core(Space &k, const void *rhs, void *x, void *r, void *rh, void *p,
                            void *v, void *sv, void *t, double target, int maxit,
                            uint64_t shadow_seed) {
    check(launch_set_target(k.sc, target, k.s));
    k.apply(x, r, false, kEpiNone, nullptr, nullptr);
    k.blas(kOpXmy, const_cast<void *>(rhs), r, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
    bicg_shadow(k, r, rh, shadow_seed);
    k.blas(kOpZero, p, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
    k.blas(kOpZero, v, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
    const int chunk = chunk_for(*k.g);
    Scalars h = read_scalars(k.sc, k.s);
    // BiCGStab's residual is not monotone; it has stagnated when its best value
    // has not improved by 1% within kStallWindow iterations.
    double best = h.rr;
    int best_it = 0;
    bool stalled = false;
    ChunkRunner runner(k.s, k.graph, chunk_key(3, k, {x, r, rh, p, v, sv, t}));
    while (!h.done && h.iter < maxit) {
        const int n = std::min(chunk, maxit - h.iter);
        runner.run(n, [&](int m) {
            for (int it = 0; it < m; ++it) {
                const int *skip = &k.sc->done;
                k.blas(kOpBiP, r, p, v);                               // p = r + b (p - w v)
                k.apply(p, v, false, kEpiBiAlpha, rh, skip);           // v = A p, alpha
                k.blas(kOpBiS, r, v, sv);                              // s = r - alpha v
                k.apply(sv, t, false, kEpiBiOmega, nullptr, skip);     // t = A s, omega
                k.blas(kOpBiXR, x, p, sv, t, r, rh, kEpiBiRho);        // x, r, rho, beta
            }
        });
        h = read_scalars(k.sc, k.s);
        if (h.rr < 0.99 * best) {
            best = h.rr;
            best_it = h.iter;
        } else if (h.iter - best_it > kStallWindow) {
            stalled = true;
            break;
        }
    }
    CoreResult res;
    res.iters = h.iter;
    res.rr = h.rr;
    res.status = h.done ? h.status : (stalled ? WL_STAGNATED : WL_NOCONV);
    return res;
}

// ---------------------------------------------------------------------------
// Mixed-precision BiCGStab with reliable updates (Sleijpen-van der Vorst): one
// BiCGStab sequence in the low-precision space klo on (r, rhat, p, v, s, t,
// x_lo). Once ||r||^2 has dropped by delta^2 since the last update (the device
// loop stops itself there, right after the x, r update of an iteration), x_lo
// is added to the FP64 solution, the residual rhs - A x is recomputed in FP64
// and replaces r, and the sequence resumes: rho = <rhat, r> of the replaced
// residual gives the direction update of that iteration, with p, v, rhat,
// alpha and omega kept. A sequence that breaks down or stalls (no 1 %
// improvement of its best residual within kStallWindow iterations) is folded
// into x as well, and the core returns to the caller, which restarts it from
// the new FP64 residual with a fresh shadow vector, as for the FP64 solve.
// ---------------------------------------------------------------------------
struct BiLoVecs {
    void *r, *rh, *p, *v, *s, *t, *x;
};

// residual reduction between reliable updates (WL_DELTA_BI_F32 / _F16 override)
static double reliable_delta_bicg(int prec) {
    const char *v = std::getenv(prec == WL_F16S ? "WL_DELTA_BI_F16" : "WL_DELTA_BI_F32");
    const double d = v ? std::atof(v) : 0.0;
    if (d > 0.0 && d < 1.0) return d;
    return prec == WL_F16S ? 0.3 : 0.1;
}

static CoreResult bicg_reliable(Space &k64, Space &klo, const void *rhs, void *x, void *r64,
                                const BiLoVecs &lo, double target, double delta, int maxit,
                                uint64_t shadow_seed) {
    const int npar = k64.npar();
    const int chunk = chunk_for(*k64.g);
    // r64 = rhs - A x in FP64; returns ||r64||^2
    auto residual64 = [&]() {
        k64.apply(x, r64, false, kEpiNone, nullptr, nullptr);
        k64.blas(kOpXmy, const_cast<void *>(rhs), r64, nullptr, nullptr, nullptr, nullptr,
                 kEpiNone, false);
        return read_scalars(k64.sc, k64.s).sums[0];
    };
    // r_lo = r64, x_lo = 0, and the device stop point delta^2 ||r||^2
    auto reload = [&](double rr) {
        check(launch_convert_spinor(*k64.g, npar, WL_F64, r64, klo.prec, lo.r, k64.s));
        klo.blas(kOpZero, lo.x, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
        check(launch_set_target(klo.sc, std::max(target, delta * delta * rr), klo.s));
    };
    CoreResult res{0, WL_NOCONV, 0.0, 0};
    double rr = residual64();
    res.rr = rr;
    if (!std::isfinite(rr)) {
        res.status = WL_BREAKDOWN;
        return res;
    }
    if (rr <= target) {
        res.status = WL_OK;
        return res;
    }
    // a fresh sequence: rhat = r (or a pseudo-random shadow), p = v = 0
    reload(rr);
    bicg_shadow(klo, lo.r, lo.rh, shadow_seed);
    klo.blas(kOpZero, lo.p, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
    klo.blas(kOpZero, lo.v, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
    int its = 0, stale = 0;
    ChunkRunner runner(klo.s, klo.graph,
                       chunk_key(4, klo, {lo.r, lo.rh, lo.p, lo.v, lo.s, lo.t, lo.x}));
    while (its < maxit) {
        Scalars h = read_scalars(klo.sc, klo.s);
        double best = h.rr;
        int best_it = h.iter;
        bool stalled = false;
        while (!h.done && its + h.iter < maxit) {
            const int n = std::min(chunk, maxit - its - h.iter);
            runner.run(n, [&](int m) {
                for (int it = 0; it < m; ++it) {
                    const int *skip = &klo.sc->done;
                    klo.blas(kOpBiP, lo.r, lo.p, lo.v);
                    klo.apply(lo.p, lo.v, false, kEpiBiAlpha, lo.rh, skip);
                    klo.blas(kOpBiS, lo.r, lo.v, lo.s);
                    klo.apply(lo.s, lo.t, false, kEpiBiOmega, nullptr, skip);
                    klo.blas(kOpBiXR, lo.x, lo.p, lo.s, lo.t, lo.r, lo.rh, kEpiBiRho);
                }
            });
            h = read_scalars(klo.sc, klo.s);
            if (h.rr < 0.99 * best) {
                best = h.rr;
                best_it = h.iter;
            } else if (h.iter - best_it > kStallWindow) {
                stalled = true;
                break;
            }
        }
        its += h.iter;
        // reliable update: x += x_lo in FP64, the FP64 residual replaces r
        check(launch_accum_lo(*k64.g, npar, klo.prec, lo.x, x, k64.s));
        const double rr_new = residual64();
        res.updates += 1;
        res.rr = rr_new;
        if (!std::isfinite(rr_new)) {
            res.status = WL_BREAKDOWN;
            break;
        }
        if (rr_new <= target) {
            res.status = WL_OK;
            break;
        }
        if (stalled) {
            res.status = WL_STAGNATED;
            break;
        }
        if (!h.done || h.status != WL_OK) {   // out of iterations, or broken down
            res.status = h.done ? h.status : WL_NOCONV;
            break;
        }
        stale = rr_new < 0.5 * rr ? 0 : stale + 1;
        if (stale > 8) {
            res.status = WL_STAGNATED;
            break;
        }
        rr = rr_new;
        reload(rr);
        klo.blas(kOpNormDot, lo.rh, lo.r, nullptr, nullptr, nullptr, nullptr, kEpiBiResume,
                 false);
    }
    res.iters = its;
    return res;
}

// ---------------------------------------------------------------------------
// Even-odd source preparation and reconstruction (in the space's precision)
// ---------------------------------------------------------------------------
// bhat_e = b_e + kappa D_eo b_o  (twisted mass: b_e + kappa D_eo A^-1 b_o,
// with A^-1 b_o formed in the space's intermediate block)
static void eo_source(Space &k, const void *b_full, void *bhat_e) {
    HopCall c{};
    c.gauge = k.gauge;
    c.in[1] = k.par(b_full, 1);
    if (k.tw != 0.0) {
        Space one = k;
        one.eo = true;   // one parity block per field
        one.blas(kOpTwist, const_cast<void *>(k.par(b_full, 1)), k.tmp, nullptr, nullptr,
                 nullptr, nullptr, kEpiNone, false, 1.0 / (1.0 + k.tw * k.tw), -k.tw);
        c.in[1] = k.tmp;
    }
    c.xs[0] = b_full;
    c.out[0] = bhat_e;
    c.first_par = 0; c.npar = 1; c.dag = false;
    c.nrhs = k.nrhs; c.fstride = k.fstride;
    k.coef(c, 1.0, 1);
    check(launch_hop(*k.g, k.prec, k.link12, k.ph, c, k.s));
}

// x_o = b_o + kappa D_oe x_e   (x_full's even block holds x_e)
static void eo_reconstruct(Space &k, const void *b_full, void *x_full) {
    HopCall c{};
    c.gauge = k.gauge;
    c.in[0] = x_full;
    c.xs[1] = k.par(b_full, 1);
    c.out[1] = k.par(x_full, 1);
    c.first_par = 1; c.npar = 1; c.dag = false;
    c.nrhs = k.nrhs; c.fstride = k.fstride;
    k.coef(c, 1.0, 1);
    if (k.tw != 0.0) {   // x_o = A^-1 (b_o + kappa D_oe x_e)
        const double s = 1.0 / (1.0 + k.tw * k.tw);
        c.c *= s;
        c.sx = s;
        c.tx = c.ta = -k.tw;
    }
    check(launch_hop(*k.g, k.prec, k.link12, k.ph, c, k.s));
}

// ||b - M x||^2 in FP64 on the full lattice; leaves b - M x in `res`
static double true_res2(Space &k64full, const void *b, const void *x, void *res) {
    k64full.apply(x, res, false, kEpiNone, nullptr, nullptr);
    k64full.blas(kOpXmy, const_cast<void *>(b), res, nullptr, nullptr, nullptr, nullptr,
                 kEpiNone, false);
    return read_scalars(k64full.sc, k64full.s).sums[0];
}

// ---------------------------------------------------------------------------
// Model cost per Krylov iteration (flops: 1320 per site per hopping term plus
// 48 per xpay; bytes: compulsory traffic of every kernel)
// ---------------------------------------------------------------------------
struct Cost {
    double flops, bytes;
};

// bytes of one stored spinor site and one stored link
static double site_bytes(int prec) { return prec == WL_F64 ? 192.0 : prec == WL_F32 ? 96.0 : 52.0; }
static double link_bytes(int prec, bool link12) {
    return (prec == WL_F64 ? 16.0 : prec == WL_F32 ? 8.0 : 4.0) * (link12 ? 6 : 9);
}

static Cost apply_cost(const Geom &g, int prec, bool link12, bool eo) {
    const double V = 2.0 * g.Vh;
    const double sp = site_bytes(prec);
    const double ln = link_bytes(prec, link12);
    if (!eo) return {1368.0 * V, V * (2 * sp + 4 * ln)};
    // two half hops over V/2 sites each; the second adds the xpay read
    return {(2 * 1320.0 + 48.0) * V / 2, V / 2 * (2 * (2 * sp + 8 * ln) + sp)};
}

static Cost iter_cost(const Geom &g, int prec, bool link12, bool eo, bool bicg,
                      bool fused = false) {
    const Cost a = apply_cost(g, prec, link12, eo);
    const double Vs = eo ? g.Vh : 2.0 * g.Vh;
    const double sp = site_bytes(prec);
    // CG: 2 applies + CgXR (4 reads, 2 writes) + CgP (2 reads, 1 write); with
    // the update fused into the adjoint (Space::cg_step) q is neither written
    // nor read again. BiCGStab: 2 applies (+1 aux read) + BiP (3r 1w) + BiS
    // (2r 1w) + BiXR (5r 2w)
    const double vec = bicg ? (1 + 4 + 3 + 7) : (fused ? 4 + 3 : 6 + 3);
    return {2 * a.flops, 2 * a.bytes + vec * Vs * sp};
}

// ---------------------------------------------------------------------------
// Driver
// ---------------------------------------------------------------------------

constexpr int kMaxRestarts = 40;

// WL_GRAPH solves run on the library's stream once the caller's stream has
// drained; returns false (and sets why) when that fails.
static bool graph_setup(SolveIn &in, std::string *why) {
    if (!(in.flags & WL_GRAPH) || in.own_stream) return true;
    hipError_t e = hipStreamSynchronize(in.s);
    if (e == hipSuccess) {
        try {
            in.s = graph_stream();
        } catch (const Fail &f) {
            e = f.err;
        }
    }
    if (e != hipSuccess) *why = std::string("HIP error preparing graph replay: ") + hipGetErrorString(e);
    return e == hipSuccess;
}

int run_solver(bool bicg, const SolveIn &in0, wl_solve_stats *st, std::string *why) {
    const auto t0 = std::chrono::steady_clock::now();
    SolveIn in = in0;
    const PageableStatus pageable(in.no_alloc);
    if (!graph_setup(in, why)) return WL_EHIP;
    const bool graph = in.flags & WL_GRAPH;
    const Geom &g = in.g;
    const bool eo = in.flags & WL_EO;
    const bool link12 = in.flags & WL_LINK12;
    const bool mixed = in.flags & WL_MIXED;
    Workspace ws = carve(g, in.flags, in.work);

    Space full64{&g, WL_F64, link12, in.ph, in.gauge, in.kappa, false, in.s, ws.sc,
                 ws.partials, nullptr};
    full64.tw = 2.0 * in.kappa * in.mu;
    wl_solve_stats out{};
    double flops = 0, bytes = 0;
    int status = WL_NOCONV;
    try {
        if (!(in.flags & WL_X0))
            full64.blas(kOpZero, in.x, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
        const double b2 = full64.norm2(in.b);
        bytes += 2.0 * g.Vh * 192.0;
        if (!(b2 > 0.0)) {
            if (!std::isfinite(b2)) {
                *why = "b is not finite";
                status = WL_BREAKDOWN;
            } else {   // b = 0: x = 0 is exact
                full64.blas(kOpZero, in.x, nullptr, nullptr, nullptr, nullptr, nullptr,
                            kEpiNone, false);
                status = WL_OK;
            }
            check(hipStreamSynchronize(in.s));
        } else {
            const double tol2 = in.tol * in.tol * b2;
            const Cost tr = apply_cost(g, WL_F64, link12, false);
            double r2 = true_res2(full64, in.b, in.x, ws.v64[6]);
            flops += tr.flops;
            bytes += tr.bytes + 3.0 * 2 * g.Vh * 192.0;
            int total_it = 0, restarts = 0, reliable = 0, fp64_it = 0;
            double best_r2 = r2;
            int since_best = 0;

            // Krylov on the caller's x (even block for eo): plain FP64, or
            // low-precision iterations with reliable FP64 updates (mixed)
            Space k{&g, WL_F64, link12, in.ph, in.gauge, in.kappa, eo, in.s, ws.sc,
                    ws.partials, ws.v64[7]};
            const int lo = lo_prec(in.flags);
            Space k32{&g, lo, link12, in.ph, ws.gauge32, in.kappa, eo, in.s, ws.sc,
                      ws.partials, ws.v32[7]};
            k.graph = k32.graph = graph;
            k.tw = k32.tw = full64.tw;
            if (mixed)
                check(launch_convert_gauge(g, link12, in.gauge, lo, ws.gauge32, in.s));
            void *rhs = const_cast<void *>(in.b);
            if (eo) {
                eo_source(k, in.b, ws.v64[5]);
                rhs = ws.v64[5];
            }
            double mb2 = 0;
            if (!bicg) {   // ||A^dag rhs||^2 sets the scale of the CG target
                k.apply(rhs, ws.v64[2], true, kEpiNone, nullptr, nullptr);
                mb2 = k.norm2(ws.v64[2]);
            }
            const double rhs2 = bicg ? k.norm2(rhs) : 0.0;
            double eta = in.tol;
            // a mixed BiCGStab whose low-precision sequence stops making
            // progress continues in FP64 from its best iterate
            bool fp64_bicg = false;
            // a BiCGStab pass that broke down without any progress is tried
            // again from the same iterate with a pseudo-random shadow vector
            // instead of rhat = r (a Krylov scalar vanished or overflowed for
            // that shadow); a few such retries in a row are allowed
            uint64_t shadow_seed = 0;
            int breakdowns = 0;
            const bool trace = std::getenv("WL_TRACE") != nullptr;
            while (true) {
                if (r2 <= tol2) { status = WL_OK; break; }
                if (total_it >= in.maxiter) { status = WL_NOCONV; break; }
                if (mixed && bicg && !fp64_bicg && since_best > 3) {
                    fp64_bicg = true;
                    since_best = 0;
                }
                if (restarts > kMaxRestarts || since_best > 3) { status = WL_STAGNATED; break; }
                // keep the current iterate: if this Krylov pass leaves x
                // worse (a stalled BiCGStab), the solve returns this one
                full64.blas(kOpCopy, in.x, ws.v64[8], nullptr, nullptr, nullptr, nullptr,
                            kEpiNone, false);
                const double r2_prev = r2;
                CoreResult cr;
                const int left = in.maxiter - total_it;
                bool lo_iters = mixed;
                if (bicg && (!mixed || fp64_bicg)) {
                    cr = bicg_core(k, rhs, in.x, ws.v64[0], ws.v64[1], ws.v64[2],
                                   ws.v64[3], ws.v64[4], ws.v64[6], eta * eta * rhs2, left,
                                   shadow_seed);
                    lo_iters = false;
                    if (mixed) fp64_it += cr.iters;
                } else if (bicg) {
                    const BiLoVecs lv{ws.v32[0], ws.v32[1], ws.v32[2], ws.v32[3],
                                      ws.v32[4], ws.v32[5], ws.v32[6]};
                    cr = bicg_reliable(k, k32, rhs, in.x, ws.v64[0], lv, eta * eta * rhs2,
                                       reliable_delta_bicg(lo), left, shadow_seed);
                } else if (mixed) {
                    const LoVecs lv{ws.v32[0], ws.v32[1], ws.v32[2], ws.v32[3], ws.v32[6]};
                    cr = cg_reliable(k, k32, rhs, in.x, ws.v64[0], ws.v64[2], lv,
                                     eta * eta * mb2, reliable_delta(lo), left);
                } else {
                    cr = cg_core(k, rhs, in.x, ws.v64[0], ws.v64[1], ws.v64[2], ws.v64[3],
                                 eta * eta * mb2, left);
                }
                if (lo_iters) {   // cost of the FP64 residual replacements
                    const Cost u = apply_cost(g, WL_F64, link12, eo);
                    const double Vs = eo ? g.Vh : 2.0 * g.Vh;
                    const double napply = bicg ? 1 : 2;
                    flops += cr.updates * napply * u.flops;
                    bytes += cr.updates * (napply * u.bytes +
                                           Vs * (6 * 192.0 + 3 * site_bytes(lo)));
                    reliable += cr.updates;
                }
                total_it += cr.iters;
                const int iprec = lo_iters ? lo : WL_F64;
                const Cost c = iter_cost(g, iprec, link12, eo, bicg,
                                         !bicg && Space::fuses_cg(eo));
                flops += c.flops * cr.iters;
                bytes += c.bytes * cr.iters;
                if (eo) eo_reconstruct(k, in.b, in.x);
                r2 = true_res2(full64, in.b, in.x, ws.v64[6]);
                flops += tr.flops;
                bytes += tr.bytes + 5.0 * 2 * g.Vh * 192.0;
                if (trace)
                    std::fprintf(stderr, "[wl] %s pass %d (%s%s): %d iterations, %d updates, "
                                 "core status %d, true residual %.3e -> %.3e\n",
                                 bicg ? "bicgstab" : "cg", restarts,
                                 lo_iters ? "low precision" : "fp64",
                                 shadow_seed ? ", random shadow" : "", cr.iters, cr.updates,
                                 cr.status, std::sqrt(r2_prev / b2), std::sqrt(r2 / b2));
                if (!(r2 < r2_prev)) {   // no progress: restore the kept iterate
                    full64.blas(kOpCopy, ws.v64[8], in.x, nullptr, nullptr, nullptr, nullptr,
                                kEpiNone, false);
                    r2 = true_res2(full64, in.b, in.x, ws.v64[6]);
                    flops += tr.flops;
                    bytes += tr.bytes + 5.0 * 2 * g.Vh * 192.0;
                    if (mixed && bicg && !fp64_bicg && std::isfinite(r2)) {
                        fp64_bicg = true;   // go on in FP64 from the kept iterate
                        since_best = 0;
                        ++restarts;
                        continue;
                    }
                    if (bicg && cr.status == WL_BREAKDOWN && breakdowns < 3 &&
                        std::isfinite(r2)) {
                        // retry from the kept iterate with a pseudo-random shadow
                        ++breakdowns;
                        shadow_seed = 0x5eed0000ull + uint64_t(restarts) + 1;
                        ++restarts;
                        continue;
                    }
                    status = !std::isfinite(r2) ? WL_BREAKDOWN
                           : (cr.status == WL_BREAKDOWN ? WL_BREAKDOWN : WL_STAGNATED);
                    if (r2 <= tol2) status = WL_OK;
                    break;
                }
                breakdowns = 0;   // progress: the next pass restarts with rhat = r
                shadow_seed = 0;
                if (r2 < best_r2 * 0.5) { best_r2 = r2; since_best = 0; }
                else ++since_best;
                if (!std::isfinite(r2)) { status = WL_BREAKDOWN; break; }
                if (r2 <= tol2) { status = WL_OK; break; }
                ++restarts;
                if (cr.status != WL_BREAKDOWN) {
                    const double rho = std::sqrt(r2 / b2);
                    eta = std::max(eta * (in.tol / rho) * 0.5, 1e-17);
                }
            }
            out.iterations = total_it;
            out.fp64_iterations = mixed ? fp64_it : total_it;
            out.restarts = restarts;
            out.reliable_updates = reliable;
            out.true_res = std::sqrt(r2 / b2);
        }
        check(hipStreamSynchronize(in.s));
    } catch (const Fail &f) {
        *why = std::string("HIP error in solver: ") + hipGetErrorString(f.err);
        (void)hipStreamSynchronize(in.s);   // drain; the first error is the one reported
        status = WL_EHIP;
    }
    const auto t1 = std::chrono::steady_clock::now();
    out.status = status;
    out.seconds = std::chrono::duration<double>(t1 - t0).count();
    out.flops = flops;
    out.bytes = bytes;
    if (st) *st = out;
    return status;
}

// ---------------------------------------------------------------------------
// Batched CGNR: nrhs right-hand sides on one lattice, solved together (the 12
// spin-colour point sources of one propagator are such a batch). Every kernel
// of an iteration covers all RHS, with the RHS index fastest in the block
// order, so each link is fetched from HBM once per site and re-served from L2
// to the other RHS. Each RHS owns a Scalars block: its own alpha, beta, stop
// flag and target, so it stops on its own; true residuals and restarts are
// per RHS as in the single solve.
// ---------------------------------------------------------------------------
static size_t batch_header_bytes(const Geom &g, int nrhs) {
    return align_up(size_t(nrhs) * sizeof(Scalars) + 4096) +
           align_up(sizeof(double) * kMaxSums * 2 * size_t(g.bpp) * nrhs);
}

// low-precision fields per RHS of a mixed batched solve: r, p, t, q, x_lo and
// the even-odd intermediate
constexpr int kVecBatchLo = 6;

size_t workspace_bytes_batch(const Geom &g, uint32_t flags, int nrhs, bool own_gauges) {
    size_t n = batch_header_bytes(g, nrhs) +
               kVecBatch * size_t(nrhs) * align_up(2 * spinor_block_bytes(g, WL_F64));
    if (flags & WL_MIXED) {
        const int lo = lo_prec(flags);
        n += kVecBatchLo * size_t(nrhs) * align_up(2 * spinor_block_bytes(g, lo)) +
             size_t(own_gauges ? nrhs : 1) * align_up(gauge_bytes(g, lo, flags & WL_LINK12)) +
             align_up(size_t(nrhs) * sizeof(void *));
    }
    return n;
}

static void read_scalars_n(const Scalars *dev, int n, hipStream_t s, Scalars *out) {
    Scalars *h = host_scalars();
    check(hipMemcpyAsync(h, dev, sizeof(Scalars) * n, hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    std::memcpy(out, h, sizeof(Scalars) * n);
}

static void norm2_n(Space &k, const void *v, double *out) {
    k.blas(kOpNorm2, const_cast<void *>(v), nullptr, nullptr, nullptr, nullptr, nullptr,
           kEpiNone, false);
    Scalars h[kMaxBatch];
    read_scalars_n(k.sc, k.nrhs, k.s, h);
    for (int r = 0; r < k.nrhs; ++r) out[r] = h[r].sums[0];
}

// CG iterations for every RHS until each meets its own target (or maxit)
static void cg_core_batch(Space &k, const void *rhs, void *x, void *r, void *p, void *t, void *q,
                          const double *targets, int maxit, int *iters) {
    check(launch_set_targets(k.sc, targets, k.nrhs, k.s));
    k.apply(x, t, false, kEpiNone, nullptr, nullptr);
    k.blas(kOpXmy, const_cast<void *>(rhs), t, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
    k.apply(t, r, true, kEpiNone, nullptr, nullptr);
    k.blas(kOpCopyNorm2, r, p, nullptr, nullptr, nullptr, nullptr, kEpiCgInit, false);
    const int chunk = chunk_for(*k.g);
    Scalars h[kMaxBatch];
    read_scalars_n(k.sc, k.nrhs, k.s, h);
    auto all_done = [&]() {
        for (int i = 0; i < k.nrhs; ++i)
            if (!h[i].done && h[i].iter < maxit) return false;
        return true;
    };
    int done_it = 0;
    ChunkRunner runner(k.s, k.graph, chunk_key(5, k, {x, r, p, t, q}));
    int len = chunk;
    double rr0[kMaxBatch];
    int it0[kMaxBatch];
    while (!all_done() && done_it < maxit) {
        const int n = std::min(len, maxit - done_it);
        for (int i = 0; i < k.nrhs; ++i) {
            rr0[i] = h[i].rr;
            it0[i] = h[i].iter;
        }
        runner.run(n, [&](int m) {
            for (int it = 0; it < m; ++it) {
                const int *skip = &k.sc->done;
                k.apply(p, t, false, kEpiCgPap, nullptr, skip);
                k.cg_step(t, q, x, p, r, skip);
                k.blas(kOpCgP, r, p);
            }
        });
        done_it += n;
        read_scalars_n(k.sc, k.nrhs, k.s, h);
        // the slowest unconverged RHS sets the next chunk (a full one when
        // any of them has no estimate)
        double need = 0.0;
        for (int i = 0; i < k.nrhs; ++i) {
            if (h[i].done) continue;
            const double ni = cg_need(rr0[i], h[i].iter - it0[i], h[i]);
            if (ni < 0.0) {
                need = -1.0;
                break;
            }
            need = std::max(need, ni);
        }
        len = next_chunk(chunk, need);
    }
    for (int i = 0; i < k.nrhs; ++i) iters[i] = h[i].iter;
}

// Mixed-precision CGNR with reliable updates for every RHS of a batch: the
// per-RHS sequence of cg_reliable (low-precision iterations until the residual
// has dropped by delta^2, or has not halved in kInnerStall iterations, then an
// FP64 residual replacement), with all RHS iterating in the same batched
// launches. An RHS that reaches its stop point idles (its kernels skip) until
// every RHS has; the replacements then run together. Per RHS the operations
// are those of the single solve, so each solution keeps its single-solve bits.
struct BatchLo {
    void *r, *p, *t, *q, *x;
    size_t fs;   // field stride of the low-precision batch vectors
};

static Space one_rhs(const Space &k, int r) {
    Space o = k;
    o.nrhs = 1;
    o.sc = k.sc + r;
    return o;
}

static void *field(void *base, size_t fs, int r) { return static_cast<char *>(base) + r * fs; }

static void cg_reliable_batch(Space &k64, Space &k32, const void *rhs, void *x, void *r64,
                              void *t64, const BatchLo &lo, const double *targets, double delta,
                              int maxit, int *iters, int *updates, int *status) {
    const int n = k64.nrhs;
    const int npar = k64.npar();
    const Geom &g = *k64.g;
    const int chunk = chunk_for(g);
    const size_t fs64 = k64.fstride;
    std::vector<double> rr(n), rr_new(n), tg(n), best(n);
    std::vector<int> its(n, 0), stale(n, 0), best_it(n), stopped(n);
    std::vector<char> active(n, 0);
    auto residual64 = [&](std::vector<double> &out) {
        k64.apply(x, t64, false, kEpiNone, nullptr, nullptr);
        k64.blas(kOpXmy, const_cast<void *>(rhs), t64, nullptr, nullptr, nullptr, nullptr,
                 kEpiNone, false);
        k64.apply(t64, r64, true, kEpiNone, nullptr, nullptr);
        norm2_n(k64, r64, out.data());
    };
    auto reload = [&]() {
        for (int r = 0; r < n; ++r)
            if (active[r])
                check(launch_convert_spinor(g, npar, WL_F64, field(r64, fs64, r), k32.prec,
                                            field(lo.r, lo.fs, r), k64.s));
        k32.blas(kOpZero, lo.x, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
        for (int r = 0; r < n; ++r)
            tg[r] = active[r] ? std::max(targets[r], delta * delta * rr[r]) : HUGE_VAL;
        check(launch_set_targets(k32.sc, tg.data(), n, k32.s));
    };
    residual64(rr);
    for (int r = 0; r < n; ++r) {
        iters[r] = updates[r] = 0;
        status[r] = WL_NOCONV;
        if (!std::isfinite(rr[r])) status[r] = WL_BREAKDOWN;
        else if (rr[r] <= targets[r]) status[r] = WL_OK;
        else active[r] = 1;
    }
    if (std::find(active.begin(), active.end(), 1) == active.end()) return;
    reload();
    k32.blas(kOpCopyNorm2, lo.r, lo.p, nullptr, nullptr, nullptr, nullptr, kEpiCgInit, false);
    Scalars h[kMaxBatch];
    ChunkRunner runner(k32.s, k32.graph, chunk_key(6, k32, {lo.p, lo.t, lo.q, lo.x, lo.r}));
    while (true) {
        read_scalars_n(k32.sc, n, k32.s, h);
        auto running = [&](int r) { return active[r] && !h[r].done && its[r] + h[r].iter < maxit; };
        for (int r = 0; r < n; ++r) {
            best[r] = h[r].rr;
            best_it[r] = h[r].iter;
            stopped[r] = 0;
        }
        int len = chunk;
        while (true) {
            int m = 0;
            for (int r = 0; r < n; ++r)
                if (running(r)) m = std::max(m, 1);
            if (!m) break;
            int steps = len;
            for (int r = 0; r < n; ++r)
                if (running(r)) steps = std::min(steps, maxit - its[r] - h[r].iter);
            double rr0[kMaxBatch];
            int it0[kMaxBatch];
            for (int r = 0; r < n; ++r) {
                rr0[r] = h[r].rr;
                it0[r] = h[r].iter;
            }
            runner.run(steps, [&](int cnt) {
                for (int it = 0; it < cnt; ++it) {
                    const int *skip = &k32.sc->done;
                    k32.apply(lo.p, lo.t, false, kEpiCgPap, nullptr, skip);
                    k32.cg_step(lo.t, lo.q, lo.x, lo.p, lo.r, skip);
                    k32.blas(kOpCgP, lo.r, lo.p);
                }
            });
            read_scalars_n(k32.sc, n, k32.s, h);
            for (int r = 0; r < n; ++r) {
                if (!active[r] || h[r].done) continue;
                bool stop = false;
                if (h[r].rr < 0.5 * best[r]) {
                    best[r] = h[r].rr;
                    best_it[r] = h[r].iter;
                } else if (h[r].iter - best_it[r] > kInnerStall) {
                    stop = true;   // at the inner precision's noise floor
                }
                if (its[r] + h[r].iter >= maxit) stop = true;
                if (stop) {
                    stopped[r] = 1;
                    check(launch_stop_rhs(k32.sc + r, k32.s));
                }
            }
            for (int r = 0; r < n; ++r)
                if (stopped[r]) h[r].done = 1;   // mirrors the device flag just set
            // the next chunk: as in cg_core_batch, for the RHS still iterating
            double need = 0.0;
            for (int r = 0; r < n; ++r) {
                if (!running(r)) continue;
                const double nr = cg_need(rr0[r], h[r].iter - it0[r], h[r]);
                if (nr < 0.0) {
                    need = -1.0;
                    break;
                }
                need = std::max(need, nr);
            }
            len = next_chunk(chunk, need);
        }
        // reliable update of every RHS that iterated in this cycle
        for (int r = 0; r < n; ++r) {
            if (!active[r]) continue;
            its[r] += h[r].iter;
            check(launch_accum_lo(g, npar, k32.prec, field(lo.x, lo.fs, r), field(x, fs64, r),
                                  k64.s));
        }
        residual64(rr_new);
        bool any = false;
        for (int r = 0; r < n; ++r) {
            if (!active[r]) continue;
            updates[r] += 1;
            if (!std::isfinite(rr_new[r])) {
                status[r] = WL_BREAKDOWN;
                active[r] = 0;
            } else if (rr_new[r] <= targets[r]) {
                status[r] = WL_OK;
                active[r] = 0;
            } else {
                stale[r] = rr_new[r] < 0.5 * rr[r] ? 0 : stale[r] + 1;
                if (stale[r] > 8) {
                    status[r] = WL_STAGNATED;
                    active[r] = 0;
                } else if (its[r] >= maxit) {
                    status[r] = WL_NOCONV;
                    active[r] = 0;
                } else {
                    rr[r] = rr_new[r];
                    any = true;
                }
            }
        }
        if (!any) break;
        reload();
        k32.blas(kOpNorm2, lo.r, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiCgInit, false);
        for (int r = 0; r < n; ++r) {
            if (!active[r]) continue;
            Space o = one_rhs(k32, r);
            void *lr = field(lo.r, lo.fs, r), *lp = field(lo.p, lo.fs, r);
            if (!stopped[r] && h[r].done && h[r].status == WL_OK && h[r].beta > 0.0 && h[r].rr > 0.0) {
                check(launch_beta_ratio(k32.sc + r, h[r].rr / h[r].beta, k32.s));
                o.blas(kOpCgP, lr, lp, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
            } else {
                o.blas(kOpCopy, lr, lp, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
            }
        }
    }
    for (int r = 0; r < n; ++r) iters[r] = its[r];
}

int run_cg_batch(const SolveIn &in0, int nrhs, wl_solve_stats *st, std::string *why) {
    const auto t0 = std::chrono::steady_clock::now();
    SolveIn in = in0;
    if (!graph_setup(in, why)) return WL_EHIP;
    const Geom &g = in.g;
    const bool eo = in.flags & WL_EO;
    const bool link12 = in.flags & WL_LINK12;
    const size_t fs = align_up(2 * spinor_block_bytes(g, WL_F64));   // == the caller's stride
    char *base = static_cast<char *>(in.work);
    Scalars *sc = reinterpret_cast<Scalars *>(base);
    double *partials = reinterpret_cast<double *>(
        base + align_up(size_t(nrhs) * sizeof(Scalars) + 4096));
    char *v[kVecBatch];
    char *p = base + batch_header_bytes(g, nrhs);
    for (int i = 0; i < kVecBatch; ++i, p += fs * nrhs) v[i] = p;

    Space full{&g, WL_F64, link12, in.ph, in.gauge, in.kappa, false, in.s, sc, partials, nullptr};
    full.nrhs = nrhs;
    full.fstride = fs;
    Space k{&g, WL_F64, link12, in.ph, in.gauge, in.kappa, eo, in.s, sc, partials, v[7]};
    k.nrhs = nrhs;
    k.fstride = fs;
    k.graph = in.flags & WL_GRAPH;
    full.gtab = k.gtab = in.gtab;
    full.per_kappa = k.per_kappa = in.kappas != nullptr;

    // mixed precision: low-precision batch vectors, gauge copies and table
    const bool mixed = in.flags & WL_MIXED;
    const int lo = lo_prec(in.flags);
    const bool own_gauges = in.gtab != nullptr;
    BatchLo lov{};
    Space k32 = k;
    if (mixed) {
        lov.fs = align_up(2 * spinor_block_bytes(g, lo));
        void **lv[5] = {&lov.r, &lov.p, &lov.t, &lov.q, &lov.x};
        for (int i = 0; i < 5; ++i, p += lov.fs * nrhs) *lv[i] = p;
        void *tmp32 = p;
        p += lov.fs * nrhs;
        const size_t gb = align_up(gauge_bytes(g, lo, link12));
        char *g32 = p;
        p += gb * (own_gauges ? nrhs : 1);
        const void **gtab32 = reinterpret_cast<const void **>(p);
        k32 = Space{&g, lo, link12, in.ph, g32, in.kappa, eo, in.s, sc, partials, tmp32};
        k32.nrhs = nrhs;
        k32.fstride = lov.fs;
        k32.graph = k.graph;
        k32.per_kappa = k.per_kappa;
        try {
            if (own_gauges) {
                if (!in.gauges_host) throw Fail{hipErrorInvalidValue};
                std::vector<const void *> t32(nrhs);
                for (int r = 0; r < nrhs; ++r) {
                    t32[r] = g32 + r * gb;
                    check(launch_convert_gauge(g, link12, in.gauges_host[r], lo,
                                               const_cast<void *>(t32[r]), in.s));
                }
                check(hipMemcpyAsync(gtab32, t32.data(), nrhs * sizeof(void *),
                                     hipMemcpyHostToDevice, in.s));
                check(hipStreamSynchronize(in.s));
                k32.gtab = gtab32;
            } else {
                check(launch_convert_gauge(g, link12, in.gauge, lo, g32, in.s));
            }
        } catch (const Fail &f) {
            *why = std::string("HIP error preparing the mixed batch: ") + hipGetErrorString(f.err);
            return WL_EHIP;
        }
    }
    std::vector<int> updates(nrhs, 0), upd(nrhs, 0), core_status(nrhs, 0);

    std::vector<double> b2(nrhs), r2(nrhs), mb2(nrhs), eta(nrhs, in.tol), targets(nrhs);
    std::vector<int> iters(nrhs, 0), total(nrhs, 0), restarts(nrhs, 0), status(nrhs, WL_NOCONV);
    std::vector<int> since_best(nrhs, 0);
    std::vector<double> best(nrhs);
    double flops = 0, bytes = 0;
    int ret = WL_OK;
    const Cost tr = apply_cost(g, WL_F64, link12, false);
    const int iprec = (in.flags & WL_MIXED) ? lo_prec(in.flags) : WL_F64;
    const Cost ic = iter_cost(g, iprec, link12, eo, false, Space::fuses_cg(eo));
    auto true_res = [&]() {
        full.apply(in.x, v[6], false, kEpiNone, nullptr, nullptr);
        full.blas(kOpXmy, const_cast<void *>(in.b), v[6], nullptr, nullptr, nullptr, nullptr,
                  kEpiNone, false);
        Scalars h[kMaxBatch];
        read_scalars_n(sc, nrhs, in.s, h);
        for (int r = 0; r < nrhs; ++r) r2[r] = h[r].sums[0];
        flops += nrhs * tr.flops;
        bytes += nrhs * (tr.bytes + 3.0 * 2 * g.Vh * 192.0);
    };
    try {
        if (in.kappas) check(launch_set_kappas(sc, in.kappas, nrhs, in.s));
        if (!(in.flags & WL_X0))
            full.blas(kOpZero, in.x, nullptr, nullptr, nullptr, nullptr, nullptr, kEpiNone, false);
        norm2_n(full, in.b, b2.data());
        true_res();
        void *rhs = const_cast<void *>(in.b);
        if (eo) {
            eo_source(k, in.b, v[5]);
            rhs = v[5];
        }
        k.apply(rhs, v[2], true, kEpiNone, nullptr, nullptr);
        norm2_n(k, v[2], mb2.data());
        std::vector<char> active(nrhs, 1);
        for (int r = 0; r < nrhs; ++r) {
            best[r] = r2[r];
            if (b2[r] == 0.0) {   // b = 0: x = 0 is exact
                Space one = full;
                one.nrhs = 1;
                one.sc = sc + r;
                one.blas(kOpZero, static_cast<char *>(in.x) + r * fs, nullptr, nullptr, nullptr,
                         nullptr, nullptr, kEpiNone, false);
                r2[r] = 0.0;
                status[r] = WL_OK;
                active[r] = 0;
            }
        }
        while (true) {
            bool any = false;
            for (int r = 0; r < nrhs; ++r) {
                if (!active[r]) continue;
                const double tol2 = in.tol * in.tol * b2[r];
                int s = -1;
                if (!std::isfinite(b2[r]) || !std::isfinite(r2[r])) s = WL_BREAKDOWN;
                else if (r2[r] <= tol2) s = WL_OK;
                else if (total[r] >= in.maxiter) s = WL_NOCONV;
                else if (restarts[r] > kMaxRestarts || since_best[r] > 3) s = WL_STAGNATED;
                if (s >= 0) {
                    status[r] = s;
                    active[r] = 0;
                } else {
                    any = true;
                }
            }
            if (!any) break;
            int left = 0;
            for (int r = 0; r < nrhs; ++r) {
                // an RHS that is finished gets a target it already meets: its kernels idle
                targets[r] = active[r] ? eta[r] * eta[r] * mb2[r] : HUGE_VAL;
                if (active[r]) left = std::max(left, in.maxiter - total[r]);
            }
            if (mixed) {
                cg_reliable_batch(k, k32, rhs, in.x, v[0], v[2], lov, targets.data(),
                                  reliable_delta(lo), left, iters.data(), upd.data(),
                                  core_status.data());
                const Cost u = apply_cost(g, WL_F64, link12, eo);
                const double Vs = eo ? g.Vh : 2.0 * g.Vh;
                for (int r = 0; r < nrhs; ++r) {
                    updates[r] += upd[r];
                    flops += upd[r] * 2 * u.flops;
                    bytes += upd[r] * (2 * u.bytes + Vs * (6 * 192.0 + 3 * site_bytes(lo)));
                }
            } else {
                cg_core_batch(k, rhs, in.x, v[0], v[1], v[2], v[3], targets.data(), left,
                              iters.data());
            }
            for (int r = 0; r < nrhs; ++r) {
                total[r] += iters[r];
                flops += ic.flops * iters[r];
                bytes += ic.bytes * iters[r];
            }
            if (eo) eo_reconstruct(k, in.b, in.x);
            true_res();
            for (int r = 0; r < nrhs; ++r) {
                if (!active[r]) continue;
                if (r2[r] < 0.5 * best[r]) { best[r] = r2[r]; since_best[r] = 0; }
                else ++since_best[r];
                if (r2[r] > in.tol * in.tol * b2[r]) {
                    ++restarts[r];
                    const double rho = std::sqrt(r2[r] / b2[r]);
                    eta[r] = std::max(eta[r] * (in.tol / rho) * 0.5, 1e-17);
                }
            }
        }
        check(hipStreamSynchronize(in.s));
    } catch (const Fail &f) {
        *why = std::string("HIP error in solver: ") + hipGetErrorString(f.err);
        (void)hipStreamSynchronize(in.s);   // drain; the first error is the one reported
        for (int r = 0; r < nrhs; ++r) status[r] = WL_EHIP;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < nrhs; ++r) {
        if (st) {
            st[r] = wl_solve_stats{};
            st[r].status = status[r];
            st[r].iterations = total[r];
            st[r].fp64_iterations = mixed ? 0 : total[r];
            st[r].restarts = restarts[r];
            st[r].reliable_updates = updates[r];
            st[r].true_res = b2[r] > 0.0 ? std::sqrt(r2[r] / b2[r]) : 0.0;
            st[r].seconds = secs;
            st[r].flops = flops / nrhs;
            st[r].bytes = bytes / nrhs;
        }
        if (status[r] < 0) ret = status[r];
        else if (ret == WL_OK) ret = status[r];
    }
    return ret;
}

// ---------------------------------------------------------------------------
// Uneven batches of independent problems (lattices of several sizes, each
// with its own gauge field and kappa). Problems of one size form a group
// solved as one batched CG (per-RHS gauge table and kappa); the groups run
// concurrently, each on its own host thread and its own stream, so the GPU
// overlaps the small lattices. Sources are copied into the group's contiguous
// batch and solutions copied back.
// ---------------------------------------------------------------------------
constexpr size_t kMaxGroupThreads = 8;

struct Group {
    Geom g;
    std::vector<int> idx;
    size_t off;
};

size_t problem_group_bytes(const Geom &g, uint32_t flags, int m) {
    const size_t fs = align_up(2 * spinor_block_bytes(g, WL_F64));
    return align_up(size_t(m) * sizeof(void *)) + 2 * size_t(m) * fs +
           workspace_bytes_batch(g, flags, m, true);
}

// m problems of one lattice size solved as one batch on stream s: sources are
// gathered into a batch in `work` (problem_group_bytes(g, flags, m) bytes),
// the batched CG runs with each problem's gauge field and kappa, and the
// solutions are scattered back. Every problem's result is bitwise its solo one.
int run_problem_group(const wl_problem *const *p, int m, const Geom &g, const Phases &ph,
                      double tol, int maxiter, uint32_t flags, void *work, hipStream_t s,
                      wl_solve_stats *st, std::string *why) {
    const size_t fs = align_up(2 * spinor_block_bytes(g, WL_F64));
    const size_t fbytes = 2 * spinor_block_bytes(g, WL_F64);
    try {
        char *base = static_cast<char *>(work);
        const void **gtab = reinterpret_cast<const void **>(base);
        char *bb = base + align_up(size_t(m) * sizeof(void *));
        char *xb = bb + m * fs;
        void *ws = xb + m * fs;
        std::vector<const void *> ptrs(m);
        std::vector<double> kap(m);
        for (int r = 0; r < m; ++r) {
            ptrs[r] = p[r]->gauge;
            kap[r] = p[r]->kappa;
            check(hipMemcpyAsync(bb + r * fs, p[r]->b, fbytes, hipMemcpyDeviceToDevice, s));
            if (flags & WL_X0)
                check(hipMemcpyAsync(xb + r * fs, p[r]->x, fbytes, hipMemcpyDeviceToDevice, s));
        }
        check(hipMemcpyAsync(gtab, ptrs.data(), m * sizeof(void *), hipMemcpyHostToDevice, s));
        check(hipStreamSynchronize(s));
        SolveIn in{};
        in.gauge = ptrs[0];
        in.b = bb;
        in.x = xb;
        in.g = g;
        in.kappa = kap[0];
        in.ph = ph;
        in.tol = tol;
        in.maxiter = maxiter;
        in.flags = flags;
        in.work = ws;
        in.s = s;
        in.gtab = gtab;
        in.gauges_host = ptrs.data();
        in.kappas = kap.data();
        in.own_stream = true;
        const int status = run_cg_batch(in, m, st, why);
        for (int r = 0; r < m; ++r)
            check(hipMemcpyAsync(p[r]->x, xb + r * fs, fbytes, hipMemcpyDeviceToDevice, s));
        check(hipStreamSynchronize(s));
        return status;
    } catch (const Fail &f) {
        (void)hipStreamSynchronize(s);
        *why = std::string("HIP error in problem batch: ") + hipGetErrorString(f.err);
    } catch (const std::exception &e) {
        (void)hipStreamSynchronize(s);
        *why = std::string("host error in problem batch: ") + e.what();
    }
    for (int r = 0; r < m; ++r) {
        st[r] = wl_solve_stats{};
        st[r].status = WL_EHIP;
    }
    return WL_EHIP;
}

static std::vector<Group> plan_groups(const wl_problem *p, int n, uint32_t flags, size_t *total,
                                      std::string *why) {
    std::vector<Group> gs;
    size_t off = 0;
    std::vector<char> used(n, 0);
    for (int i = 0; i < n; ++i) {
        if (used[i]) continue;
        Geom g;
        if (!make_geom(p[i].dims, &g, why)) return {};
        std::vector<int> same;
        for (int j = i; j < n; ++j)
            if (!used[j] && std::memcmp(p[j].dims, p[i].dims, sizeof(p[i].dims)) == 0) {
                same.push_back(j);
                used[j] = 1;
            }
        for (size_t a = 0; a < same.size(); a += kMaxBatch) {
            Group gr;
            gr.g = g;
            gr.idx.assign(same.begin() + a, same.begin() + std::min(same.size(), a + kMaxBatch));
            gr.off = off;
            off += problem_group_bytes(g, flags, int(gr.idx.size()));
            gs.push_back(gr);
        }
    }
    *total = off;
    return gs;
}

size_t problems_workspace_bytes(const wl_problem *p, int n, uint32_t flags) {
    size_t total = 0;
    std::string why;
    plan_groups(p, n, flags, &total, &why);
    return total;
}

int run_problems(const wl_problem *p, int n, const Phases &ph, double tol, int maxiter,
                 uint32_t flags, void *work, hipStream_t caller, wl_solve_stats *st,
                 std::string *why) {
    size_t total = 0;
    std::vector<Group> gs = plan_groups(p, n, flags, &total, why);
    if (gs.empty()) return WL_EINVAL;
    if (hipStreamSynchronize(caller) != hipSuccess) {
        *why = "caller stream failed";
        return WL_EHIP;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *why = "hipGetDevice failed";
        return WL_EHIP;
    }
    std::vector<int> gstatus(gs.size(), WL_OK);
    std::vector<std::string> gwhy(gs.size());
    std::vector<std::vector<wl_solve_stats>> gst(gs.size());
    auto work_group = [&](size_t gi) {
        const Group &gr = gs[gi];
        const int m = int(gr.idx.size());
        gst[gi].assign(m, wl_solve_stats{});
        std::vector<const wl_problem *> ps(m);
        for (int r = 0; r < m; ++r) ps[r] = &p[gr.idx[r]];
        hipStream_t s = nullptr;
        if (hipSetDevice(dev) != hipSuccess ||   // the device is per host thread
            hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            gstatus[gi] = WL_EHIP;
            gwhy[gi] = "HIP error creating the problem batch's stream";
            return;
        }
        gstatus[gi] = run_problem_group(ps.data(), m, gr.g, ph, tol, maxiter, flags,
                                        static_cast<char *>(work) + gr.off, s, gst[gi].data(),
                                        &gwhy[gi]);
        (void)hipStreamDestroy(s);
    };
    // a small pool of host threads takes the groups in order
    std::atomic<size_t> next{0};
    auto worker = [&]() {
        for (size_t gi; (gi = next.fetch_add(1)) < gs.size();) work_group(gi);
    };
    const size_t nthreads = std::min<size_t>(gs.size(), kMaxGroupThreads);
    std::vector<std::thread> threads;
    for (size_t t = 1; t < nthreads; ++t) threads.emplace_back(worker);
    worker();
    for (auto &t : threads) t.join();
    int ret = WL_OK;
    for (size_t gi = 0; gi < gs.size(); ++gi) {
        for (size_t r = 0; r < gs[gi].idx.size(); ++r)
            if (st) st[gs[gi].idx[r]] = gst[gi][r];
        if (gstatus[gi] != WL_OK && (ret == WL_OK || gstatus[gi] < 0)) {
            ret = gstatus[gi];
            *why = gwhy[gi];
        }
    }
    return ret;
}

}  // namespace wl
