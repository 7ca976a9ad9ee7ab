// wl_internal.h -- shared declarations of libwilson.so (not installed).
//
// Geometry of the even-odd ("WL") layout, the complex type used in kernels,
// vector-chunk loads and stores, the solver scalar block, and the launchers
// each .hip file provides to the host-side drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>

#include "wilson.h"

namespace wl {

constexpr int kBlock = 256;      // threads per block of every site kernel
constexpr int kMaxSums = 4;      // doubles per fused reduction

// ---------------------------------------------------------------------------
// Lattice geometry of the packed layout
// ---------------------------------------------------------------------------
struct Geom {
    int L[4];   // extents x, y, z, t
    int Lxh;    // Lx / 2
    int Vh;     // sites per parity
    int S;      // parity-block stride in sites (Vh rounded up to 64)
    int bpp;    // blocks of kBlock threads per parity
};

bool make_geom(const int32_t dims[4], Geom *g, std::string *why);

// ---------------------------------------------------------------------------
// Complex numbers in kernels
// ---------------------------------------------------------------------------
template <typename R>
struct cpx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <typename R>
__device__ __forceinline__ cpx<R> ci(cpx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.re, -a.im}; }

// ---------------------------------------------------------------------------
// Storage chunks: a field of NC complex numbers per site is stored as NC/CW
// arrays of vectors holding CW complex numbers each, one array per chunk,
// each of length S (sites of one parity).
// ---------------------------------------------------------------------------
template <typename R, int CW> struct Vec;
template <> struct Vec<double, 1> { using T = double2; };
template <> struct Vec<float, 1> { using T = float2; };
template <> struct Vec<float, 2> { using T = float4; };

template <typename R>
struct SpinorFmt {
    static constexpr int CW = std::is_same<R, double>::value ? 1 : 2;
    static constexpr int NCH = 12 / CW;   // chunks per site
    using T = typename Vec<R, CW>::T;
};

template <typename R, int NCL>   // NCL = 9 (18-real) or 6 (12-real)
struct LinkFmt {
    static constexpr int CW = (std::is_same<R, double>::value || NCL == 9) ? 1 : 2;
    static constexpr int NCH = NCL / CW;
    using T = typename Vec<R, CW>::T;
};

template <typename R, int NC, int CW>
__device__ __forceinline__ void load_cplx(const typename Vec<R, CW>::T *__restrict__ p,
                                          int S, int i, cpx<R> *v) {
#pragma unroll
    for (int j = 0; j < NC / CW; ++j) {
        const typename Vec<R, CW>::T c = p[j * S + i];
        if constexpr (CW == 1) {
            v[j].re = c.x;
            v[j].im = c.y;
        } else {
            v[2 * j].re = c.x;
            v[2 * j].im = c.y;
            v[2 * j + 1].re = c.z;
            v[2 * j + 1].im = c.w;
        }
    }
}

template <typename R, int NC, int CW>
__device__ __forceinline__ void store_cplx(typename Vec<R, CW>::T *__restrict__ p,
                                           int S, int i, const cpx<R> *v) {
#pragma unroll
    for (int j = 0; j < NC / CW; ++j) {
        typename Vec<R, CW>::T c;
        if constexpr (CW == 1) {
            c.x = v[j].re;
            c.y = v[j].im;
        } else {
            c.x = v[2 * j].re;
            c.y = v[2 * j].im;
            c.z = v[2 * j + 1].re;
            c.w = v[2 * j + 1].im;
        }
        p[j * S + i] = c;
    }
}

// one site of a spinor parity block
template <typename R>
__device__ __forceinline__ void load_spinor(const void *blk, int S, int i, cpx<R> v[12]) {
    using F = SpinorFmt<R>;
    load_cplx<R, 12, F::CW>(static_cast<const typename F::T *>(blk), S, i, v);
}
template <typename R>
__device__ __forceinline__ void store_spinor(void *blk, int S, int i, const cpx<R> v[12]) {
    using F = SpinorFmt<R>;
    store_cplx<R, 12, F::CW>(static_cast<typename F::T *>(blk), S, i, v);
}

// Byte sizes
size_t spinor_block_bytes(const Geom &g, int prec);   // one parity block
size_t gauge_bytes(const Geom &g, int prec, bool link12);

// ---------------------------------------------------------------------------
// Deterministic fused reductions
// ---------------------------------------------------------------------------
// Every reducing kernel writes one partial per block per sum into `partials`
// ([sum][block]); the last block to finish (counted on `counter`) adds the
// partials in a fixed order, writes the totals, runs the epilogue, and resets
// the counter to zero. The totals therefore do not depend on block timing.
struct Reduce {
    double *partials;     // kMaxSums * max_blocks doubles
    unsigned *counter;    // zero between launches
    double *result;       // kMaxSums doubles (may alias scalars)
    int epilogue;         // Epi::*
    struct Scalars *sc;   // solver state the epilogue updates
};

enum Epi : int {
    kEpiNone = 0,
    kEpiCgInit,     // sum0 = ||r||^2 of a fresh residual
    kEpiCgPap,      // sum0 = ||M p||^2 = <p, M^dag M p>
    kEpiCgRr,       // sum0 = ||r_new||^2
    kEpiBiInit,     // sum0 = ||r||^2 (rhat = r, rho = ||r||^2)
    kEpiBiAlpha,    // sum0,1 = <rhat, v>
    kEpiBiOmega,    // sum0,1 = <t, s>, sum2 = <t, t>
    kEpiBiRho,      // sum0 = ||r||^2, sum1,2 = <rhat, r>
};

// Solver state in device memory (lives at the start of the workspace).
struct Scalars {
    double rr;          // current ||r||^2 (recursive)
    double target;      // stop when rr <= target
    double pap;         // CG: ||M p||^2
    double alpha;       // CG step
    double beta;        // CG direction update
    double rho[2];      // BiCGStab rho (complex)
    double alpha_c[2];  // BiCGStab alpha (complex)
    double omega[2];    // BiCGStab omega (complex)
    double beta_c[2];   // BiCGStab beta (complex)
    double sums[kMaxSums];   // totals of the last reduction
    int done;           // 1 once converged or broken down: kernels become no-ops
    int iter;           // Krylov iterations since the last (re)start
    int status;         // WL_OK or WL_BREAKDOWN
    int pad;
};

// ---------------------------------------------------------------------------
// Launchers (host side)
// ---------------------------------------------------------------------------
struct Phases {
    double re[4], im[4];
};

// out[p] = (xs ? xs[p] : 0) + c * D_{p,1-p} in[1-p] for the output parities
// p in {first_par, ...} (npar = 1 or 2). Optional fused ||out||^2 reduction.
struct HopCall {
    const void *gauge;
    const void *in[2];
    const void *xs[2];
    const void *aux[2];   // <aux, out> operand (BiCGStab alpha); else null
    void *out[2];
    int first_par;
    int npar;
    double c;
    bool dag;
    const int *skip;      // kernel is a no-op when *skip != 0 (may be null)
    const Reduce *red;    // null: no reduction
};
hipError_t launch_hop(const Geom &g, int prec, bool link12, const Phases &ph,
                      const HopCall &call, hipStream_t s);

// Canonical complex128 <-> packed
hipError_t launch_pack_gauge(const Geom &g, int prec, bool link12, const void *canon,
                             void *packed, hipStream_t s);
hipError_t launch_pack_spinor(const Geom &g, int prec, const void *canon, void *packed,
                              hipStream_t s);
hipError_t launch_unpack_spinor(const Geom &g, int prec, const void *packed, void *canon,
                                hipStream_t s);
// Packed FP64 <-> FP32 conversions (npar parity blocks of spinors; gauge)
hipError_t launch_convert_spinor(const Geom &g, int npar, int src_prec, const void *src,
                                 int dst_prec, void *dst, hipStream_t s);
hipError_t launch_convert_gauge(const Geom &g, bool link12, const void *src64, void *dst32,
                                hipStream_t s);

// ---- BLAS-1 on packed spinor fields of npar parity blocks ----------------
enum BlasOp : int {
    kOpZero = 0,        // y = 0
    kOpCopy,            // y = x
    kOpNorm2,           // sum0 = ||x||^2
    kOpXmy,             // y = x - y                        (+ ||y||^2)
    kOpCgXR,            // x += alpha p; r -= alpha q (alpha from sc)   (+ ||r||^2)
    kOpCgP,             // p = r + beta p (beta from sc)
    kOpBiP,             // p = r + beta (p - omega v)
    kOpBiS,             // s = r - alpha v
    kOpBiXR,            // x += alpha p + omega s; r = s - omega t  (+ ||r||^2, <rhat, r>)
    kOpAxpy,            // y += a x (a = host scalar)
    kOpCopyNorm2,       // y = x, sum0 = ||x||^2 (init of CG/BiCGStab)
    kOpCopy2Norm2,      // y = x, z = x, sum0 = ||x||^2
};
struct BlasCall {
    int op;
    int npar;
    void *v[6];           // operand parity-0 blocks, meaning per op
    double a;             // host scalar for kOpAxpy
    Scalars *sc;
    const int *skip;
    const Reduce *red;
};
hipError_t launch_blas(const Geom &g, int prec, const BlasCall &call, hipStream_t s);

// Convert an FP32 half or full field and accumulate into FP64: y64 += x32
hipError_t launch_accum_f32(const Geom &g, int npar, const void *x32, void *y64,
                            hipStream_t s);

// Initialise a Krylov loop's scalars: target, done = 0, status = WL_OK, iter = 0
hipError_t launch_set_target(Scalars *sc, double target, hipStream_t s);

// ---- solvers ---------------------------------------------------------------
size_t workspace_bytes(const Geom &g, uint32_t flags);

struct SolveIn {
    const void *gauge, *b;
    void *x;
    Geom g;
    double kappa;
    Phases ph;
    double tol;
    int maxiter;
    uint32_t flags;
    void *work;
    hipStream_t s;
};

int run_solver(bool bicg, const SolveIn &in, wl_solve_stats *st, std::string *why);

}  // namespace wl
