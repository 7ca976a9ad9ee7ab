// wl_dslash.hip -- the Wilson hopping term on the even-odd layout.
//
// One thread computes one output site x of parity p:
//
//   out(x) = xs(x) + c * sum_mu [ f (1 -/+ gamma_mu) U_mu(x)        psi(x+mu)
//                               + b (1 +/- gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
//
// (paper Sec. 3: the "dslash", the non-diagonal part of the fermion matrix; the
// upper signs are D_W, the lower ones its gamma_5 conjugate D_W^dag). All eight
// neighbours have parity 1-p. Each hop first projects the neighbour spinor to
// a half spinor (two colour vectors), multiplies both by the link (or its
// adjoint), multiplies by the boundary phase when the hop wraps, and expands
// back to four spins while accumulating. Spin projection in the chiral basis
// gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_t = [[0, 1], [1, 0]]:
//   (1 + s gamma_mu) psi = (h0, h1, lower)   with, for s = +-1,
//   mu=x: h = (psi0 - s i psi3, psi1 - s i psi2), lower = (s i h1, s i h0)
//   mu=y: h = (psi0 - s psi3,   psi1 + s psi2),   lower = (s h1, -s h0)
//   mu=z: h = (psi0 - s i psi2, psi1 + s i psi3), lower = (s i h0, -s i h1)
//   mu=t: h = (psi0 + s psi2,   psi1 + s psi3),   lower = (s h0, s h1)
// Links are stored as 18 reals, or as rows 0 and 1 (12 reals) with row 2
// rebuilt as conj(row0 x row1); phases are applied after the rebuild.
// Storage is FP64, FP32 or FP16 (spinors with a per-site scale); arithmetic
// is FP64 for FP64 storage and FP32 otherwise.
//
// Model cost: 1320 flop per output site for the hopping term, +48 for the
// xpay; compulsory bytes: 8 links and 8 neighbour spinors amortised over the
// lattice (see the layout notes in wilson.h).
#include "wl_internal.h"
#include "wl_reduce.h"

// Launch-shape knobs (compile time). Minimum waves per SIMD the register
// allocation must allow, per precision; streaming (non-temporal) output
// stores; XCD-contiguous block order; interleaving the two parities' blocks
// in full-lattice launches so the blocks that share links run on one XCD.
#ifndef WL_F64_WAVES
#define WL_F64_WAVES 1
#endif
#ifndef WL_F32_WAVES
#define WL_F32_WAVES 1
#endif
#ifndef WL_NT_STORE
#define WL_NT_STORE 1
#endif
#ifndef WL_XCD_REMAP
#define WL_XCD_REMAP 1
#endif
#ifndef WL_PAR_INTERLEAVE
#define WL_PAR_INTERLEAVE 1
#endif

namespace wl {

template <typename ST>
struct MinWaves {
    static constexpr int value = std::is_same<ST, double>::value ? WL_F64_WAVES : WL_F32_WAVES;
};

enum RedMode : int { kRedNone = 0, kRedNorm = 1, kRedDotAux = 2, kRedTS = 3 };

template <typename R>
struct HopArgs {
    const void *gauge;     // packed gauge base (parity 0, mu 0, chunk 0)
    const void *in[2];     // input parity blocks
    const void *xs[2];     // xpay source parity blocks (or null)
    const void *aux[2];    // vector for <aux, out> (kRedDotAux)
    void *out[2];          // output parity blocks
    Geom g;
    int first_par;         // parity of the first output block
    int npar;              // output parities in this launch (1 or 2)
    int nblocks;           // nb_rhs * nrhs
    int nb_rhs;            // blocks per right-hand side
    int nrhs;              // right-hand sides (fields fstride bytes apart)
    size_t fstride;
    R c;
    R phr[4], phi[4];      // boundary phases
    const int *skip;
    Reduce red;
    const void *const *gtab;   // per-RHS gauge fields (or null: `gauge` shared)
    const Scalars *ksc;        // per-RHS kappa (or null: `c` shared)
    R cmul;
    int cpow;
};

template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cpx<R> psi[12], cpx<R> h[6]) {
    // psi[spin*3 + colour]
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<R> p0 = psi[a], p1 = psi[3 + a], p2 = psi[6 + a], p3 = psi[9 + a];
        if constexpr (MU == 0) {
            h[a] = (S > 0) ? p0 - ci(p3) : p0 + ci(p3);
            h[3 + a] = (S > 0) ? p1 - ci(p2) : p1 + ci(p2);
        } else if constexpr (MU == 1) {
            h[a] = (S > 0) ? p0 - p3 : p0 + p3;
            h[3 + a] = (S > 0) ? p1 + p2 : p1 - p2;
        } else if constexpr (MU == 2) {
            h[a] = (S > 0) ? p0 - ci(p2) : p0 + ci(p2);
            h[3 + a] = (S > 0) ? p1 + ci(p3) : p1 - ci(p3);
        } else {
            h[a] = (S > 0) ? p0 + p2 : p0 - p2;
            h[3 + a] = (S > 0) ? p1 + p3 : p1 - p3;
        }
    }
}

template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(cpx<R> acc[12], const cpx<R> u[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<R> u0 = u[a], u1 = u[3 + a];
        acc[a] = acc[a] + u0;
        acc[3 + a] = acc[3 + a] + u1;
        if constexpr (MU == 0) {
            acc[6 + a] = (S > 0) ? acc[6 + a] + ci(u1) : acc[6 + a] - ci(u1);
            acc[9 + a] = (S > 0) ? acc[9 + a] + ci(u0) : acc[9 + a] - ci(u0);
        } else if constexpr (MU == 1) {
            acc[6 + a] = (S > 0) ? acc[6 + a] + u1 : acc[6 + a] - u1;
            acc[9 + a] = (S > 0) ? acc[9 + a] - u0 : acc[9 + a] + u0;
        } else if constexpr (MU == 2) {
            acc[6 + a] = (S > 0) ? acc[6 + a] + ci(u0) : acc[6 + a] - ci(u0);
            acc[9 + a] = (S > 0) ? acc[9 + a] - ci(u1) : acc[9 + a] + ci(u1);
        } else {
            acc[6 + a] = (S > 0) ? acc[6 + a] + u0 : acc[6 + a] - u0;
            acc[9 + a] = (S > 0) ? acc[9 + a] + u1 : acc[9 + a] - u1;
        }
    }
}

template <typename ST, int NCL>
__device__ __forceinline__ void load_link(const void *gauge, const Geom &g, int par, int mu,
                                          int i, cpx<Real<ST>> u[9]) {
    load_link_raw<ST, NCL>(gauge, g.S, par, mu, i, u);
    if constexpr (NCL == 6) {
        u[6] = cconj(u[1] * u[5] - u[2] * u[4]);
        u[7] = cconj(u[2] * u[3] - u[0] * u[5]);
        u[8] = cconj(u[0] * u[4] - u[1] * u[3]);
    }
}

// u h (forward) on both colour vectors of the half spinor
template <typename R>
__device__ __forceinline__ void su3_mul(const cpx<R> u[9], const cpx<R> h[6], cpx<R> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            o[3 * sp + a] = u[3 * a] * h[3 * sp] + u[3 * a + 1] * h[3 * sp + 1] +
                            u[3 * a + 2] * h[3 * sp + 2];
}

// u^dag h (backward)
template <typename R>
__device__ __forceinline__ void su3_dag_mul(const cpx<R> u[9], const cpx<R> h[6], cpx<R> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            o[3 * sp + a] = cmulc(u[a], h[3 * sp]) + cmulc(u[3 + a], h[3 * sp + 1]) +
                            cmulc(u[6 + a], h[3 * sp + 2]);
}

template <typename R>
__device__ __forceinline__ void times_phase(cpx<R> o[6], R pr, R pi) {
    const cpx<R> ph{pr, pi};
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = ph * o[k];
}

// One hop direction: forward (FWD) or backward, projector sign S.
template <typename ST, int NCL, int MU, int S, bool FWD>
__device__ __forceinline__ void hop_dir(const HopArgs<Real<ST>> &a, const void *gauge,
                                        const void *in_blk, int p, int i, int nb, bool wrap,
                                        cpx<Real<ST>> acc[12]) {
    using R = Real<ST>;
    cpx<R> psi[12];
    load_spinor<ST>(in_blk, a.g.S, nb, psi);
    cpx<R> h[6];
    project<MU, S>(psi, h);
    cpx<R> u[9];
    cpx<R> o[6];
    if constexpr (FWD) {
        load_link<ST, NCL>(gauge, a.g, p, MU, i, u);
        su3_mul(u, h, o);
        if (wrap) times_phase(o, a.phr[MU], a.phi[MU]);
    } else {
        load_link<ST, NCL>(gauge, a.g, 1 - p, MU, nb, u);
        su3_dag_mul(u, h, o);
        if (wrap) times_phase(o, a.phr[MU], -a.phi[MU]);
    }
    accumulate<MU, S>(acc, o);
}

template <typename ST, int NCL, bool DAG, bool XPAY, int RED>
__global__ void __launch_bounds__(kBlock, MinWaves<ST>::value) hop_kernel(HopArgs<Real<ST>> a) {
    using R = Real<ST>;
    const Geom &g = a.g;
    // logical block -> (right-hand side, block of that field); the RHS index
    // runs fastest so the blocks sharing a site range (and its links) are
    // consecutive and land on one XCD
    const int bl = WL_XCD_REMAP ? xcd_block(blockIdx.x, a.nblocks) : int(blockIdx.x);
    const int rhs = bl % a.nrhs;
    const int b = bl / a.nrhs;
    if (rhs_skip(a.skip, rhs)) return;
    const size_t fo = size_t(rhs) * a.fstride;
    const void *gauge = a.gtab ? a.gtab[rhs] : a.gauge;
    R c = a.c;
    if (a.ksc) {
        const R k = R(a.ksc[rhs].kappa);
        c = a.cpow == 2 ? a.cmul * k * k : (a.cpow == 1 ? a.cmul * k : a.cmul);
    }
    int pidx, bi;
    if (WL_PAR_INTERLEAVE && a.npar == 2) {
        pidx = b & 1;
        bi = b >> 1;
    } else {
        pidx = b >= g.bpp ? 1 : 0;
        bi = b - pidx * g.bpp;
    }
    const int p = a.first_par ^ pidx;
    const int i = bi * kBlock + threadIdx.x;

    constexpr int NS = RED == kRedNone ? 1 : (RED == kRedNorm ? 1 : (RED == kRedDotAux ? 2 : 3));
    double sums[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) sums[s] = 0.0;

    if (i < g.Vh) {
        // coordinates of the output site
        const int xh = i % g.Lxh;
        int r = i / g.Lxh;
        const int y = r % g.L[1];
        r /= g.L[1];
        const int z = r % g.L[2];
        const int t = r / g.L[2];
        const int x = 2 * xh + ((y + z + t + p) & 1);

        const void *in_blk = static_cast<const char *>(a.in[1 - p]) + fo;
        constexpr int SF = DAG ? 1 : -1;   // forward projector 1 + SF gamma
        constexpr int SB = -SF;            // backward projector 1 + SB gamma

        cpx<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};

        {   // x direction: neighbour checkerboard index changes through x/2
            const int xp = (x + 1 == g.L[0]) ? 0 : x + 1;
            const int xm = (x == 0) ? g.L[0] - 1 : x - 1;
            hop_dir<ST, NCL, 0, SF, true>(a, gauge, in_blk, p, i,i - xh + (xp >> 1), x == g.L[0] - 1, acc);
            hop_dir<ST, NCL, 0, SB, false>(a, gauge, in_blk, p, i,i - xh + (xm >> 1), x == 0, acc);
        }
        {
            const int st = g.Lxh;
            const int span = (g.L[1] - 1) * st;
            hop_dir<ST, NCL, 1, SF, true>(a, gauge, in_blk, p, i,y == g.L[1] - 1 ? i - span : i + st,
                                          y == g.L[1] - 1, acc);
            hop_dir<ST, NCL, 1, SB, false>(a, gauge, in_blk, p, i,y == 0 ? i + span : i - st, y == 0, acc);
        }
        {
            const int st = g.Lxh * g.L[1];
            const int span = (g.L[2] - 1) * st;
            hop_dir<ST, NCL, 2, SF, true>(a, gauge, in_blk, p, i,z == g.L[2] - 1 ? i - span : i + st,
                                          z == g.L[2] - 1, acc);
            hop_dir<ST, NCL, 2, SB, false>(a, gauge, in_blk, p, i,z == 0 ? i + span : i - st, z == 0, acc);
        }
        {
            const int st = g.Lxh * g.L[1] * g.L[2];
            const int span = (g.L[3] - 1) * st;
            hop_dir<ST, NCL, 3, SF, true>(a, gauge, in_blk, p, i,t == g.L[3] - 1 ? i - span : i + st,
                                          t == g.L[3] - 1, acc);
            hop_dir<ST, NCL, 3, SB, false>(a, gauge, in_blk, p, i,t == 0 ? i + span : i - st, t == 0, acc);
        }

        cpx<R> o[12];
        cpx<R> xv[12];
        if constexpr (XPAY) {
            load_spinor<ST>(static_cast<const char *>(a.xs[p]) + fo, g.S, i, xv);
#pragma unroll
            for (int k = 0; k < 12; ++k) o[k] = xv[k] + c * acc[k];
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) o[k] = c * acc[k];
        }
        store_spinor<ST, WL_NT_STORE != 0>(static_cast<char *>(a.out[p]) + fo, g.S, i, o);

        if constexpr (RED == kRedNorm) {
#pragma unroll
            for (int k = 0; k < 12; ++k)
                sums[0] += double(o[k].re) * double(o[k].re) + double(o[k].im) * double(o[k].im);
        } else if constexpr (RED == kRedDotAux) {   // <aux, out>
            cpx<R> w[12];
            load_spinor<ST>(static_cast<const char *>(a.aux[p]) + fo, g.S, i, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                sums[0] += double(w[k].re) * double(o[k].re) + double(w[k].im) * double(o[k].im);
                sums[1] += double(w[k].re) * double(o[k].im) - double(w[k].im) * double(o[k].re);
            }
        } else if constexpr (RED == kRedTS) {       // <out, xs>, ||out||^2
            static_assert(XPAY, "kRedTS needs the xpay source");
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                sums[0] += double(o[k].re) * double(xv[k].re) + double(o[k].im) * double(xv[k].im);
                sums[1] += double(o[k].re) * double(xv[k].im) - double(o[k].im) * double(xv[k].re);
                sums[2] += double(o[k].re) * double(o[k].re) + double(o[k].im) * double(o[k].im);
            }
        }
    }
    if constexpr (RED != kRedNone)
        block_partial<NS>(sums, rhs_reduce(a.red, rhs, a.nb_rhs).partials, b, a.nb_rhs);
}

template <typename ST, int NCL, bool DAG, bool XPAY, int RED>
static hipError_t launch_t(const HopArgs<Real<ST>> &a, hipStream_t s) {
    hipLaunchKernelGGL((hop_kernel<ST, NCL, DAG, XPAY, RED>), dim3(a.nblocks), dim3(kBlock), 0, s,
                       a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || RED == kRedNone) return e;
    constexpr int NS = RED == kRedNorm ? 1 : (RED == kRedDotAux ? 2 : 3);
    return launch_finish(a.red, NS, a.nb_rhs, a.nrhs, a.skip, s);
}

template <typename ST, int NCL, bool DAG, bool XPAY>
static hipError_t launch_red(const HopArgs<Real<ST>> &a, int red, hipStream_t s) {
    switch (red) {
    case kRedNone: return launch_t<ST, NCL, DAG, XPAY, kRedNone>(a, s);
    case kRedNorm: return launch_t<ST, NCL, DAG, XPAY, kRedNorm>(a, s);
    case kRedDotAux: return launch_t<ST, NCL, DAG, XPAY, kRedDotAux>(a, s);
    default:
        if constexpr (XPAY) return launch_t<ST, NCL, DAG, XPAY, kRedTS>(a, s);
        return hipErrorInvalidValue;
    }
}

template <typename ST, int NCL>
static hipError_t launch_ncl(const HopArgs<Real<ST>> &a, bool dag, bool xpay, int red,
                             hipStream_t s) {
    if (dag) {
        return xpay ? launch_red<ST, NCL, true, true>(a, red, s)
                    : launch_red<ST, NCL, true, false>(a, red, s);
    }
    return xpay ? launch_red<ST, NCL, false, true>(a, red, s)
                : launch_red<ST, NCL, false, false>(a, red, s);
}

template <typename ST>
static hipError_t launch_storage(const Geom &g, bool link12, const Phases &ph,
                                 const HopCall &call, int red, hipStream_t s) {
    using R = Real<ST>;
    HopArgs<R> a;
    a.gauge = call.gauge;
    for (int q = 0; q < 2; ++q) {
        a.in[q] = call.in[q];
        a.xs[q] = call.xs[q];
        a.out[q] = call.out[q];
        a.aux[q] = call.aux[q];
    }
    a.g = g;
    a.first_par = call.first_par;
    a.npar = call.npar;
    a.nrhs = call.nrhs < 1 ? 1 : call.nrhs;
    a.nb_rhs = g.bpp * call.npar;
    a.nblocks = a.nb_rhs * a.nrhs;
    a.fstride = call.fstride;
    a.c = R(call.c);
    for (int mu = 0; mu < 4; ++mu) {
        a.phr[mu] = R(ph.re[mu]);
        a.phi[mu] = R(ph.im[mu]);
    }
    a.skip = call.skip;
    if (call.red) a.red = *call.red;
    else a.red = Reduce{nullptr, nullptr, kEpiNone, nullptr};
    a.gtab = call.gtab;
    a.ksc = call.ksc;
    a.cmul = R(call.cmul);
    a.cpow = call.cpow;
    const bool xpay = call.xs[call.first_par] != nullptr;
    return link12 ? launch_ncl<ST, 6>(a, call.dag, xpay, red, s)
                  : launch_ncl<ST, 9>(a, call.dag, xpay, red, s);
}

hipError_t launch_hop(const Geom &g, int prec, bool link12, const Phases &ph,
                      const HopCall &call, hipStream_t s) {
    int red = kRedNone;
    if (call.red) {
        if (!call.red->partials || (!call.red->result && !call.red->sc))
            return hipErrorInvalidValue;
        red = call.red->epilogue == kEpiBiAlpha ? kRedDotAux
            : call.red->epilogue == kEpiBiOmega ? kRedTS : kRedNorm;
        if (red == kRedDotAux && !call.aux[call.first_par]) return hipErrorInvalidValue;
        if (red == kRedTS && !call.xs[call.first_par]) return hipErrorInvalidValue;
    }
    if (call.npar < 1 || call.npar > 2 || !call.out[call.first_par] ||
        !call.in[1 - call.first_par])
        return hipErrorInvalidValue;
    return with_storage(prec, [&](auto tag) {
        return launch_storage<decltype(tag)>(g, link12, ph, call, red, s);
    });
}

}  // namespace wl
