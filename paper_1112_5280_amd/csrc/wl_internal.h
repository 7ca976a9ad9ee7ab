// wl_internal.h -- shared declarations of libwilson.so (not installed).
//
// Geometry of the even-odd ("WL") layout, the complex type used in kernels,
// storage access for the three storage precisions, the solver scalar block,
// and the launchers each .hip file provides to the host-side drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>

#include "wilson.h"

namespace wl {

#ifndef WL_BLOCK
#define WL_BLOCK 256
#endif
constexpr int kBlock = WL_BLOCK; // threads per block of every site kernel (multiple of 64)
constexpr int kMaxSums = 4;      // doubles per fused reduction
constexpr int kMaxBatch = 64;    // right-hand sides per batched solve

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
// Storage precisions. ST is the storage type of a field: double, float, or
// Half (IEEE binary16; spinors carry one FP32 scale per site). Arithmetic runs
// in Real<ST>: FP64 for double storage, FP32 otherwise.
//
// A field of NC complex numbers per site is stored as NC/CW arrays ("chunks")
// of vectors of CW complex numbers, each array S sites long, so a wave's 64
// lanes read 64 consecutive sites of one chunk.
// ---------------------------------------------------------------------------
struct Half {};

template <typename ST>
using Real = typename std::conditional<std::is_same<ST, double>::value, double, float>::type;

template <typename ST>
constexpr int prec_of() {
    return std::is_same<ST, double>::value ? WL_F64 : std::is_same<ST, float>::value ? WL_F32
                                                                                      : WL_F16S;
}

// bytes of one stored complex number
template <typename ST>
constexpr int cbytes() {
    return std::is_same<ST, double>::value ? 16 : std::is_same<ST, float>::value ? 8 : 4;
}

typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

template <typename ST, int CW> struct Vec;
template <> struct Vec<double, 1> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct Vec<float, 1> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct Vec<float, 2> { typedef float T __attribute__((ext_vector_type(4))); };
template <> struct Vec<Half, 1> { typedef h2v T; };
template <> struct Vec<Half, 2> { typedef h4v T; };
template <> struct Vec<Half, 4> { typedef h8v T; };

// complex numbers per chunk: 16-byte chunks for spinors where possible
template <typename ST> constexpr int spinor_cw() { return 16 / cbytes<ST>(); }
// links: two complex per chunk for 12-real FP32/FP16 storage, else one (9 is odd)
// links: 16-byte chunks where possible (FP32 two complex, FP16 four), the
// NCL % cw complex numbers left over in one narrower tail chunk
template <typename ST, int NCL> constexpr int link_cw() {
    return std::is_same<ST, double>::value ? 1 : (std::is_same<ST, float>::value ? 2 : 4);
}

// Streaming (non-temporal) load of device memory through a global
// address-space pointer: a generic pointer would make it a flat load, which
// also occupies the scalar-memory wait counter.
template <typename T>
__device__ __forceinline__ T load_nt(const T *p) {
    typedef __attribute__((address_space(1))) const T GT;
    return __builtin_nontemporal_load((GT *)p);
}

// Element i of chunk j (S elements each) of a T array: the chunk base is
// uniform across the wave and stays in scalar registers; only the 32-bit
// byte offset of element i lives per lane, instead of a 64-bit address pair.
// S * sizeof(T) < 4 GiB (make_geom bounds the lattice).
template <typename T>
__device__ __forceinline__ const T *at32(const void *base, int j, int S, int i) {
    const char *chunk = static_cast<const char *>(base) + size_t(j) * size_t(S) * sizeof(T);
    return reinterpret_cast<const T *>(chunk + uint32_t(i) * uint32_t(sizeof(T)));
}

// NC complex numbers of site i: NC / CW arrays of S chunks of CW complex, then
// (if NC % CW != 0) one array of S chunks holding the remaining NC % CW.
// NT: read-once data (a streaming load that L2 need not keep). O32: 32-bit
// offsets (fewer address registers; it pays where registers are scarcest,
// the FP64 hopping kernels).
template <typename ST, int NC, int CW, bool NT = false, bool O32 = false>
__device__ __forceinline__ void load_cplx(const void *base, int S, int i, cpx<Real<ST>> *v) {
    using T = typename Vec<ST, CW>::T;
    using R = Real<ST>;
    constexpr int NF = NC / CW, TL = NC % CW;
    const T *p = static_cast<const T *>(base);
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        T c;
        const T *q = O32 ? at32<T>(base, j, S, i) : &p[j * S + i];
        if constexpr (NT) c = load_nt(q);
        else c = *q;
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            v[CW * j + k].re = R(c[2 * k]);
            v[CW * j + k].im = R(c[2 * k + 1]);
        }
    }
    if constexpr (TL > 0) {
        using TT = typename Vec<ST, TL>::T;
        const TT *q = reinterpret_cast<const TT *>(p + size_t(NF) * S) + i;
        TT c;
        if constexpr (NT) c = load_nt(q);
        else c = *q;
#pragma unroll
        for (int k = 0; k < TL; ++k) {
            v[CW * NF + k].re = R(c[2 * k]);
            v[CW * NF + k].im = R(c[2 * k + 1]);
        }
    }
}

template <typename ST> struct Elem { using T = ST; };
template <> struct Elem<Half> { using T = _Float16; };

template <typename ST, int NC, int CW, bool NT = false>
__device__ __forceinline__ void store_cplx(void *base, int S, int i, const cpx<Real<ST>> *v,
                                           Real<ST> scale = Real<ST>(1)) {
    using T = typename Vec<ST, CW>::T;
    using E = typename Elem<ST>::T;
    constexpr int NF = NC / CW, TL = NC % CW;
    T *p = static_cast<T *>(base);
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        T c;
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            c[2 * k] = static_cast<E>(v[CW * j + k].re * scale);
            c[2 * k + 1] = static_cast<E>(v[CW * j + k].im * scale);
        }
        if constexpr (NT) __builtin_nontemporal_store(c, &p[j * S + i]);
        else p[j * S + i] = c;
    }
    if constexpr (TL > 0) {
        using TT = typename Vec<ST, TL>::T;
        TT c;
#pragma unroll
        for (int k = 0; k < TL; ++k) {
            c[2 * k] = static_cast<E>(v[CW * NF + k].re * scale);
            c[2 * k + 1] = static_cast<E>(v[CW * NF + k].im * scale);
        }
        TT *q = reinterpret_cast<TT *>(p + size_t(NF) * S) + i;
        if constexpr (NT) __builtin_nontemporal_store(c, q);
        else *q = c;
    }
}

// ---- spinors: one site of one parity block --------------------------------
// Half blocks hold the 24 binary16 values of psi/s followed by the S scales.
// s is the power of two 2^e just above the site's largest |component| m
// (m = f 2^e, f in [0.5, 1)), so every stored value lies in (-1, 1). Scaling by
// a power of two is exact and keeps the halves' relative precision; unlike a
// reciprocal 1/m it cannot overflow when m is an FP32 denormal -- which the
// far sites of a point-source residual reach after a few iterations, since
// every hop multiplies by kappa -- and so never turns 0 * inf into NaN.
template <typename ST, bool NT = false, bool O32 = false>
__device__ __forceinline__ void load_spinor(const void *blk, int S, int i, cpx<Real<ST>> v[12]) {
    load_cplx<ST, 12, spinor_cw<ST>(), NT, O32>(blk, S, i, v);
    if constexpr (std::is_same<ST, Half>::value) {
        const float *sp = reinterpret_cast<const float *>(static_cast<const char *>(blk) +
                                                          size_t(S) * 48) + i;
        float s;
        if constexpr (NT) s = load_nt(sp);
        else s = *sp;
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = s * v[k];
    }
}

template <typename ST, bool NT = false>
__device__ __forceinline__ void store_spinor(void *blk, int S, int i, const cpx<Real<ST>> v[12]) {
    if constexpr (std::is_same<ST, Half>::value) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        int e = 0;
        (void)frexpf(m, &e);   // m = 0 gives e = 0, s = 1
        cpx<float> w[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = {ldexpf(v[k].re, -e), ldexpf(v[k].im, -e)};
        store_cplx<ST, 12, spinor_cw<ST>(), NT>(blk, S, i, w);
        reinterpret_cast<float *>(static_cast<char *>(blk) + size_t(S) * 48)[i] = ldexpf(1.f, e);
    } else {
        store_cplx<ST, 12, spinor_cw<ST>(), NT>(blk, S, i, v);
    }
}

// ---- links: U_mu at checkerboard index i of parity par --------------------
template <typename ST, int NCL>
__device__ __forceinline__ const void *link_block(const void *gauge, int S, int par, int mu) {
    return static_cast<const char *>(gauge) + size_t(par * 4 + mu) * NCL * cbytes<ST>() * S;
}

template <typename ST, int NCL, bool NT = false, bool O32 = false>
__device__ __forceinline__ void load_link_raw(const void *gauge, int S, int par, int mu, int i,
                                              cpx<Real<ST>> *u) {
    load_cplx<ST, NCL, link_cw<ST, NCL>(), NT, O32>(link_block<ST, NCL>(gauge, S, par, mu), S, i,
                                                    u);
}

template <typename ST, int NCL>
__device__ __forceinline__ void store_link_raw(void *gauge, int S, int par, int mu, int i,
                                               const cpx<Real<ST>> *u) {
    store_cplx<ST, NCL, link_cw<ST, NCL>()>(
        const_cast<void *>(link_block<ST, NCL>(gauge, S, par, mu)), S, i, u);
}

// Byte sizes
size_t spinor_block_bytes(const Geom &g, int prec);   // one parity block
size_t gauge_bytes(const Geom &g, int prec, bool link12);

// Host-side dispatch from a WL_* precision to a storage type tag.
template <typename F>
auto with_storage(int prec, F &&f) {
    if (prec == WL_F64) return f(double{});
    if (prec == WL_F32) return f(float{});
    return f(Half{});
}

// ---------------------------------------------------------------------------
// Deterministic fused reductions
// ---------------------------------------------------------------------------
// Every reducing kernel writes one partial per block per sum into `partials`
// ([rhs][sum][block]); a finish kernel (one block per RHS) adds the partials
// in a fixed order, writes the totals and runs the epilogue. The totals do not
// depend on block timing.
struct Reduce {
    double *partials;     // nrhs * kMaxSums * blocks-per-RHS doubles
    double *result;       // kMaxSums doubles per RHS (unused when sc is set)
    int epilogue;         // Epi::*
    struct Scalars *sc;   // solver state the epilogue updates (RHS r: sc[r])
};

// Add up the partials of a reducing launch (ns sums, nb blocks per RHS).
hipError_t launch_finish(const Reduce &red, int ns, int nb, int nrhs, const int *skip,
                         hipStream_t s);

enum Epi : int {
    kEpiNone = 0,
    kEpiCgInit,     // sum0 = ||r||^2 of a fresh residual
    kEpiCgPap,      // sum0 = ||M p||^2 = <p, M^dag M p>
    kEpiCgRr,       // sum0 = ||r_new||^2
    kEpiBiInit,     // sum0 = ||r||^2 (rhat = r, rho = ||r||^2)
    kEpiBiAlpha,    // sum0,1 = <rhat, v>
    kEpiBiOmega,    // sum0,1 = <t, s>, sum2 = <t, t>
    kEpiBiRho,      // sum0 = ||r||^2, sum1,2 = <rhat, r>
    kEpiBiResume,   // sum0 = ||r||^2, sum1,2 = <rhat, r> of a replaced residual
    kEpiBiInitShadow,   // sum0 = ||r||^2, sum1,2 = <rhat, r> (rhat not r)
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
    double kappa;       // hopping parameter of this problem (independent problems)
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
// p in {first_par, ...} (npar = 1 or 2). Optional fused reduction.
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
    int nrhs = 1;         // fields of a batch, fstride bytes apart (gauge shared)
    size_t fstride = 0;
    // independent problems: RHS r uses gauge gtab[r] (device array) and the
    // coefficient cmul * kappa_r^cpow with kappa_r = ksc[r].kappa
    const void *const *gtab = nullptr;
    const struct Scalars *ksc = nullptr;
    double cmul = 0.0;
    int cpow = 0;
    // twisted mass: out = sx (1 + i tx g5) xs + c (1 + i ta g5) D in
    double tx = 0.0, ta = 0.0, sx = 1.0;
    // fused CG update (one output parity, red with kEpiCgRr; one RHS per
    // thread): the hop's result q is not stored; the kernel applies
    // x += alpha p, r -= alpha q and sums ||r||^2 on the blocks cg = {x, p, r}
    // of the output parity (alpha from the RHS's Scalars). `out` stays a valid
    // buffer: the autotuner times candidate launch shapes on the plain
    // operator into it.
    void *cg[3] = {nullptr, nullptr, nullptr};
};
hipError_t launch_hop(const Geom &g, int prec, bool link12, const Phases &ph,
                      const HopCall &call, hipStream_t s);
// Device copy of bytes (a multiple of 16, 16-byte aligned) with streaming stores
hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
// The autotuner's choices so far, one line per tuned batched-operator shape.
std::string tuning_report();

// Meson correlators (wl_meson.hip): 12 packed FP64 propagator columns ->
// corr[16][Lt][2] on the device, through meson_workspace_bytes(g) of work
size_t meson_workspace_bytes(const Geom &g);
hipError_t launch_meson(const Geom &g, const void *props, int t0, double *corr, void *work,
                        hipStream_t s);

// Pure-gauge kernels (wl_gauge.hip) on the canonical complex128 field
hipError_t launch_heatbath(const Geom &g, void *canon, double beta, int nsweeps,
                           uint32_t sweep0, uint32_t seed, hipStream_t s);
size_t plaquette_workspace_bytes(const Geom &g);
hipError_t launch_plaquette(const Geom &g, const void *canon, double *out, void *work,
                            hipStream_t s);

// Canonical complex128 <-> packed
hipError_t launch_pack_gauge(const Geom &g, int prec, bool link12, const void *canon,
                             void *packed, hipStream_t s);
hipError_t launch_pack_spinor(const Geom &g, int prec, const void *canon, void *packed,
                              hipStream_t s);
hipError_t launch_unpack_spinor(const Geom &g, int prec, const void *packed, void *canon,
                                hipStream_t s);
// Packed spinor precision conversion (npar parity blocks); FP64 gauge -> lower
hipError_t launch_convert_spinor(const Geom &g, int npar, int src_prec, const void *src,
                                 int dst_prec, void *dst, hipStream_t s);
hipError_t launch_convert_gauge(const Geom &g, bool link12, const void *src64, int dst_prec,
                                void *dst, hipStream_t s);

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
    kOpNormDot,         // sum0 = ||y||^2, sum1,2 = <x, y>  (x = v0, y = v1)
    kOpRandom,          // y = pseudo-random field, components in (-1, 1), seed = a
    kOpTwist,           // y = a (1 + i b g5) x  (twisted-mass diagonal or its inverse)
};
struct BlasCall {
    int op;
    int npar;
    void *v[6];           // operand parity-0 blocks, meaning per op
    double a;             // host scalar for kOpAxpy
    double b = 0.0;       // second host scalar (kOpTwist)
    Scalars *sc;          // RHS r reads sc[r]
    const int *skip;
    const Reduce *red;
    int nrhs = 1;         // fields of a batch, fstride bytes apart
    size_t fstride = 0;
};
hipError_t launch_blas(const Geom &g, int prec, const BlasCall &call, hipStream_t s);

// y64 += x (x in FP32 or FP16 storage), npar parity blocks
hipError_t launch_accum_lo(const Geom &g, int npar, int src_prec, const void *x, void *y64,
                           hipStream_t s);

// Initialise a Krylov loop's scalars: target, done = 0, status = WL_OK, iter = 0
hipError_t launch_set_target(Scalars *sc, double target, hipStream_t s);
// CG direction update after a residual replacement: beta = sc->rr / rr_old
hipError_t launch_beta_ratio(Scalars *sc, double rr_old, hipStream_t s);
// End one RHS's Krylov loop at the current iteration (its kernels then skip)
hipError_t launch_stop_rhs(Scalars *sc, hipStream_t s);
// launch_set_target for RHS 0..n-1 of a batch (n <= kMaxBatch), host targets
hipError_t launch_set_targets(Scalars *sc, const double *targets, int n, hipStream_t s);
// sc[r].kappa = kappas[r] for r < n (n <= kMaxBatch), host values
hipError_t launch_set_kappas(Scalars *sc, const double *kappas, int n, hipStream_t s);

}  // namespace wl
