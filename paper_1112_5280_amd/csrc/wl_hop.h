// wl_hop.h -- the Wilson hopping term on the even-odd layout: kernel and
// launch templates (instantiated per storage precision in wl_hop_f64.hip,
// wl_hop_f32.hip and wl_hop_f16.hip; the autotuner lives in wl_dslash.hip).
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
// With batches of fields, a thread may own several right-hand sides (NR),
// which then share every link load.
//
// Model cost: 1320 flop per output site for the hopping term, +48 for the
// xpay; compulsory bytes: 8 links and 8 neighbour spinors amortised over the
// lattice (see the layout notes in wilson.h).
#pragma once

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

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
#ifndef WL_NT_LINKS
#define WL_NT_LINKS 1
#endif
#ifndef WL_XCD_REMAP
#define WL_XCD_REMAP 1
#endif
#ifndef WL_PAR_INTERLEAVE
#define WL_PAR_INTERLEAVE 1
#endif

namespace wl {

constexpr int kMaxNr = 4;   // right-hand sides per thread in batched launches

template <typename ST>
struct MinWaves {
    static constexpr int value = std::is_same<ST, double>::value ? WL_F64_WAVES : WL_F32_WAVES;
};

// kRedCgXR: the CG update fused into the epilogue of the adjoint's last hop
// (its output q is not stored): x += alpha p, r -= alpha q and ||r||^2
enum RedMode : int { kRedNone = 0, kRedNorm = 1, kRedDotAux = 2, kRedTS = 3, kRedCgXR = 4 };

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
    int nblocks;           // nb_rhs * ngroups
    int nb_rhs;            // blocks per right-hand side
    int ngroups;           // RHS groups (NR right-hand sides per thread)
    int chunk;             // site blocks per chunk of the block order
    int tgroup;            // slice tiles walked through time together (0: off)
    int ntile_t;           // blocks per time slice (0 when a slice is not whole blocks)
    int nrhs;              // right-hand sides (fields fstride bytes apart)
    size_t fstride;
    R c;
    R phr[4], phi[4];      // boundary phases
    const int *skip;
    Reduce red;
    const void *const *gtab;   // per-RHS gauge fields (or null: `gauge` shared)
    const Scalars *ksc;        // per-RHS kappa (or null: `c` shared)
    double cmul;
    int cpow;
    // twisted mass: out = sx (1 + i tx g5) xs + c (1 + i ta g5) acc when twist
    bool twist;
    R tx, ta, sx;
    bool lds;              // x/y neighbourhood staged in LDS (when the kernel has a window)
    void *cgv[3];          // kRedCgXR: x, p, r blocks of the output parity
};

// LDS staging of neighbour halos. A block's output sites are kBlock
// consecutive checkerboard indices; their x neighbours lie in the same rows
// and their y neighbours (except where y wraps) one row away, so all of them
// fall within Lx/2 indices of that range of the input parity block. The block
// loads this window once, with coalesced 16-byte loads, and the x and y hops
// read it from LDS; z and t neighbours (a plane or a time slice away) and
// wrapping y neighbours are read from global memory as before. Measured at
// 32^3x64: FP64 eo hop 3-4 % and full M 7-11 % faster, FP32 2-7 % and 4-8 %;
// FP16 storage gains nothing (its kernels are bound by issue, and the window
// would take LDS from its four waves per SIMD), so it has no window.
constexpr int kLdsHalo = 64;                       // largest Lx/2 staged
constexpr int kLdsWin = kBlock + 2 * kLdsHalo;     // sites of a window

// kernels with a window: one RHS per thread, FP64 or FP32 storage
template <typename ST, int NR>
constexpr bool has_window() { return NR == 1 && !std::is_same<ST, Half>::value; }
template <typename ST>
struct LdsWin {
    typedef typename Vec<ST, spinor_cw<ST>()>::T T;
    static constexpr int NCH = 12 / spinor_cw<ST>();
    T c[NCH][kLdsWin];
    float scale[std::is_same<ST, Half>::value ? kLdsWin : 1];
};

template <typename ST>
__device__ __forceinline__ void load_spinor_win(const LdsWin<ST> &w, int j,
                                                cpx<Real<ST>> v[12]) {
    using R = Real<ST>;
    constexpr int CW = spinor_cw<ST>();
#pragma unroll
    for (int ch = 0; ch < LdsWin<ST>::NCH; ++ch) {
        const typename LdsWin<ST>::T c = w.c[ch][j];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            v[CW * ch + k].re = R(c[2 * k]);
            v[CW * ch + k].im = R(c[2 * k + 1]);
        }
    }
    if constexpr (std::is_same<ST, Half>::value) {
        const float sc = w.scale[j];
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = sc * v[k];
    }
}

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

// 32-bit offset loads in the single-RHS FP64 and FP16-storage kernels
// (measured: the FP64 12-real eo hop 11 % faster, the 18-real one 4 %; no
// gain for FP32 or the register-blocked batches)
template <typename ST, int NR>
constexpr bool use_o32() { return !std::is_same<ST, float>::value && NR == 1; }

template <typename ST, int NCL, bool NTL, bool O32 = false>
__device__ __forceinline__ void load_link(const void *gauge, const Geom &g, int par, int mu,
                                          int i, cpx<Real<ST>> u[9]) {
    load_link_raw<ST, NCL, NTL, O32>(gauge, g.S, par, mu, i, u);
    if constexpr (NCL == 6) {
        u[6] = cconj(u[1] * u[5] - u[2] * u[4]);
        u[7] = cconj(u[2] * u[3] - u[0] * u[5]);
        u[8] = cconj(u[0] * u[4] - u[1] * u[3]);
    }
}

// u h (forward) on both colour vectors of the half spinor. FP32 arithmetic
// (FP32 and FP16 storage): each real component is one chain of six fmas;
// three complex products and two adds would take a multiply, five fmas and
// two adds (the FP16 kernels, bound by issue, are 9 % faster this way). FP64
// keeps the complex-product form.
template <typename R>
__device__ __forceinline__ void su3_mul(const cpx<R> u[9], const cpx<R> h[6], cpx<R> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cpx<R> *r = u + 3 * a, *v = h + 3 * sp;
            if constexpr (std::is_same<R, float>::value) {
                float re = r[0].re * v[0].re;
                re = __builtin_fmaf(-r[0].im, v[0].im, re);
                re = __builtin_fmaf(r[1].re, v[1].re, re);
                re = __builtin_fmaf(-r[1].im, v[1].im, re);
                re = __builtin_fmaf(r[2].re, v[2].re, re);
                re = __builtin_fmaf(-r[2].im, v[2].im, re);
                float im = r[0].re * v[0].im;
                im = __builtin_fmaf(r[0].im, v[0].re, im);
                im = __builtin_fmaf(r[1].re, v[1].im, im);
                im = __builtin_fmaf(r[1].im, v[1].re, im);
                im = __builtin_fmaf(r[2].re, v[2].im, im);
                im = __builtin_fmaf(r[2].im, v[2].re, im);
                o[3 * sp + a] = {re, im};
            } else {
                o[3 * sp + a] = r[0] * v[0] + r[1] * v[1] + r[2] * v[2];
            }
        }
}

// u^dag h (backward), the same two forms
template <typename R>
__device__ __forceinline__ void su3_dag_mul(const cpx<R> u[9], const cpx<R> h[6], cpx<R> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // row a of u^dag is the conjugate of column a of u
            const cpx<R> c0 = u[a], c1 = u[3 + a], c2 = u[6 + a];
            const cpx<R> *v = h + 3 * sp;
            if constexpr (std::is_same<R, float>::value) {
                float re = c0.re * v[0].re;
                re = __builtin_fmaf(c0.im, v[0].im, re);
                re = __builtin_fmaf(c1.re, v[1].re, re);
                re = __builtin_fmaf(c1.im, v[1].im, re);
                re = __builtin_fmaf(c2.re, v[2].re, re);
                re = __builtin_fmaf(c2.im, v[2].im, re);
                float im = c0.re * v[0].im;
                im = __builtin_fmaf(-c0.im, v[0].re, im);
                im = __builtin_fmaf(c1.re, v[1].im, im);
                im = __builtin_fmaf(-c1.im, v[1].re, im);
                im = __builtin_fmaf(c2.re, v[2].im, im);
                im = __builtin_fmaf(-c2.im, v[2].re, im);
                o[3 * sp + a] = {re, im};
            } else {
                o[3 * sp + a] = cmulc(c0, v[0]) + cmulc(c1, v[1]) + cmulc(c2, v[2]);
            }
        }
}

template <typename R>
__device__ __forceinline__ void times_phase(cpx<R> o[6], R pr, R pi) {
    const cpx<R> ph{pr, pi};
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = ph * o[k];
}

// One hop direction, forward (FWD) or backward, projector sign S, applied to
// the NR right-hand sides a thread owns: the link is loaded (and for 12-real
// storage rebuilt) once and multiplies the projected neighbour of every RHS.
template <typename ST, int NCL, int MU, int S, bool FWD, int NR, bool NTL, bool LW = false>
__device__ __forceinline__ void hop_dir(const HopArgs<Real<ST>> &a, const void *gauge,
                                        const char *const (&in_blk)[NR], const bool (&on)[NR],
                                        int p, int i, int nb, bool wrap,
                                        cpx<Real<ST>> (&acc)[NR][12],
                                        const LdsWin<ST> *win = nullptr, int wlo = 0,
                                        int whi = 0) {
    using R = Real<ST>;
    cpx<R> u[9];
    if constexpr (NR == 1) {
        // one RHS: neighbour spinor first, then the link (the order the
        // register allocation of the single-field kernels is best with)
        constexpr bool O32 = use_o32<ST, 1>();
        cpx<R> psi[12];
        if (LW && MU < 2 && nb >= wlo && nb < whi) load_spinor_win<ST>(*win, nb - wlo, psi);
        else load_spinor<ST, false, O32>(in_blk[0], a.g.S, nb, psi);
        cpx<R> h[6];
        project<MU, S>(psi, h);
        cpx<R> o[6];
        if constexpr (FWD) {
            load_link<ST, NCL, NTL, O32>(gauge, a.g, p, MU, i, u);
            su3_mul(u, h, o);
            if (wrap) times_phase(o, a.phr[MU], a.phi[MU]);
        } else {
            load_link<ST, NCL, NTL, O32>(gauge, a.g, 1 - p, MU, nb, u);
            su3_dag_mul(u, h, o);
            if (wrap) times_phase(o, a.phr[MU], -a.phi[MU]);
        }
        accumulate<MU, S>(acc[0], o);
        return;
    }
    if constexpr (FWD)
        load_link<ST, NCL, NTL>(gauge, a.g, p, MU, i, u);
    else
        load_link<ST, NCL, NTL>(gauge, a.g, 1 - p, MU, nb, u);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (NR > 1 && !on[r]) continue;
        cpx<R> psi[12];
        load_spinor<ST>(in_blk[r], a.g.S, nb, psi);
        cpx<R> h[6];
        project<MU, S>(psi, h);
        cpx<R> o[6];
        if constexpr (FWD) {
            su3_mul(u, h, o);
            if (wrap) times_phase(o, a.phr[MU], a.phi[MU]);
        } else {
            su3_dag_mul(u, h, o);
            if (wrap) times_phase(o, a.phr[MU], -a.phi[MU]);
        }
        accumulate<MU, S>(acc[r], o);
    }
}

// Block partials of NR right-hand sides at once: the same shuffle tree and
// wave order as block_partial, so every RHS's partial is bitwise the one a
// single-RHS launch would store.
template <int NS, int NR>
__device__ __forceinline__ void block_partial_rhs(double (&v)[NR][NS], const bool (&on)[NR],
                                                  const Reduce &red, int rhs0, int slot, int nb) {
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh[kWaves][NR][NS];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int s = 0; s < NS; ++s) v[r][s] += __shfl_xor(v[r][s], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int s = 0; s < NS; ++s) sh[wave][r][s] = v[r][s];
    __syncthreads();
    const int r = threadIdx.x;
    if (r < NR && on[r]) {
        double *partials = rhs_reduce(red, rhs0 + r, nb).partials;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += sh[w][r][s];
            partials[s * nb + slot] = t;
        }
    }
}

// NR right-hand sides per thread (register blocking over the batch). The
// logical block index runs over chunks of `chunk` consecutive site blocks;
// inside a chunk, over the RHS groups, and inside a group over the chunk's
// site blocks. chunk = 1 puts the groups that share a site range (and its
// links) back to back; a larger chunk keeps the neighbour spinors of one group
// (the z and t neighbours lie many blocks away) in cache while the next group
// still finds the chunk's links there. The order changes no arithmetic.
template <typename ST, int NCL, bool DAG, bool XPAY, int RED, int NR, bool NTL>
__global__ void __launch_bounds__(kBlock, MinWaves<ST>::value) hop_kernel(HopArgs<Real<ST>> a) {
    using R = Real<ST>;
    const Geom &g = a.g;
    const int bl = WL_XCD_REMAP ? xcd_block(blockIdx.x, a.nblocks) : int(blockIdx.x);
    const int ch = bl / (a.chunk * a.ngroups);
    const int base = ch * a.chunk;
    const int cl = min(a.chunk, a.nb_rhs - base);        // site blocks in this chunk
    const int rem = bl - base * a.ngroups;
    const int q = rem / cl;
    const int b = base + rem % cl;
    const int rhs0 = q * NR;
    bool on[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        on[r] = rhs0 + r < a.nrhs && !rhs_skip(a.skip, rhs0 + r);
        any = any || on[r];
    }
    if (!any) return;
    const void *gauge = a.gtab ? a.gtab[rhs0] : a.gauge;   // gtab only with NR = 1
    R c[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        c[r] = a.c;
        if (a.ksc) {
            // in FP64 and in the host's order, then rounded once: the
            // coefficient of a single solve with this kappa, to the bit
            const double kd = a.ksc[rhs0 + r].kappa;
            c[r] = R(a.cpow == 2 ? a.cmul * (kd * kd) : (a.cpow == 1 ? a.cmul * kd : a.cmul));
        }
    }
    int pidx, bo;   // output parity, position of the block in its parity's order
    if (WL_PAR_INTERLEAVE && a.npar == 2) {
        pidx = b & 1;
        bo = b >> 1;
    } else {
        pidx = b >= g.bpp ? 1 : 0;
        bo = b - pidx * g.bpp;
    }
    // position -> lexicographic site block bi. With tile groups (time slices
    // of a whole number of blocks), the blocks walk every time slice of
    // `tgroup` slice tiles before the next tiles: a neighbour slice is then
    // reused a few blocks later instead of a whole slice later. The partial
    // slot stays the lexicographic one, so reductions keep their bits.
    int bi = bo;
    if (a.tgroup > 0 && a.tgroup < a.ntile_t) {
        const int Lt = g.L[3];
        const int span = a.tgroup * Lt;
        const int grp = bo / span;
        const int g0 = grp * a.tgroup;
        const int gg = min(a.tgroup, a.ntile_t - g0);
        const int rem = bo - grp * span;
        bi = (rem / gg) * a.ntile_t + g0 + rem % gg;
    }
    const int slot = (WL_PAR_INTERLEAVE && a.npar == 2) ? 2 * bi + pidx : pidx * g.bpp + bi;
    const int p = a.first_par ^ pidx;
    const int i = bi * kBlock + threadIdx.x;

    constexpr bool LW = has_window<ST, NR>();
    int wlo = 0, whi = 0;
    const LdsWin<ST> *winp = nullptr;
    if constexpr (LW) {
        __shared__ LdsWin<ST> win;
        winp = &win;
        if (a.lds) {
            typedef typename LdsWin<ST>::T T;
            wlo = max(0, bi * kBlock - g.Lxh);
            whi = min(g.S, bi * kBlock + kBlock + g.Lxh);
            const char *src = static_cast<const char *>(a.in[1 - p]) + size_t(rhs0) * a.fstride;
            for (int j = threadIdx.x; j < whi - wlo; j += kBlock) {
#pragma unroll
                for (int ch = 0; ch < LdsWin<ST>::NCH; ++ch)
                    win.c[ch][j] = reinterpret_cast<const T *>(src)[size_t(ch) * g.S + wlo + j];
                if constexpr (std::is_same<ST, Half>::value)
                    win.scale[j] = reinterpret_cast<const float *>(src + size_t(g.S) * 48)[wlo + j];
            }
            __syncthreads();
        }
    }

    constexpr int NS = (RED == kRedNone || RED == kRedNorm || RED == kRedCgXR) ? 1
                     : (RED == kRedDotAux ? 2 : 3);
    double sums[NR][NS];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int s = 0; s < NS; ++s) sums[r][s] = 0.0;

    if (i < g.Vh) {
        // coordinates of the output site
        const int xh = i % g.Lxh;
        int rr = i / g.Lxh;
        const int y = rr % g.L[1];
        rr /= g.L[1];
        const int z = rr % g.L[2];
        const int t = rr / g.L[2];
        const int x = 2 * xh + ((y + z + t + p) & 1);

        size_t fo[NR];
        const char *in_blk[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            fo[r] = size_t(rhs0 + r) * a.fstride;
            in_blk[r] = static_cast<const char *>(a.in[1 - p]) + fo[r];
        }
        constexpr int SF = DAG ? 1 : -1;   // forward projector 1 + SF gamma
        constexpr int SB = -SF;            // backward projector 1 + SB gamma

        cpx<R> acc[NR][12];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[r][k] = {R(0), R(0)};

        {   // x direction: neighbour checkerboard index changes through x/2
            const int xp = (x + 1 == g.L[0]) ? 0 : x + 1;
            const int xm = (x == 0) ? g.L[0] - 1 : x - 1;
            hop_dir<ST, NCL, 0, SF, true, NR, NTL, LW>(a, gauge, in_blk, on, p, i,
                                                      i - xh + (xp >> 1), x == g.L[0] - 1, acc,
                                                      winp, wlo, whi);
            hop_dir<ST, NCL, 0, SB, false, NR, NTL, LW>(a, gauge, in_blk, on, p, i,
                                                       i - xh + (xm >> 1), x == 0, acc, winp,
                                                       wlo, whi);
        }
        {
            const int st = g.Lxh;
            const int span = (g.L[1] - 1) * st;
            hop_dir<ST, NCL, 1, SF, true, NR, NTL, LW>(a, gauge, in_blk, on, p, i,
                                                      y == g.L[1] - 1 ? i - span : i + st,
                                                      y == g.L[1] - 1, acc, winp, wlo, whi);
            hop_dir<ST, NCL, 1, SB, false, NR, NTL, LW>(a, gauge, in_blk, on, p, i,
                                                       y == 0 ? i + span : i - st, y == 0, acc,
                                                       winp, wlo, whi);
        }
        {
            const int st = g.Lxh * g.L[1];
            const int span = (g.L[2] - 1) * st;
            hop_dir<ST, NCL, 2, SF, true, NR, NTL>(a, gauge, in_blk, on, p, i,
                                              z == g.L[2] - 1 ? i - span : i + st,
                                              z == g.L[2] - 1, acc);
            hop_dir<ST, NCL, 2, SB, false, NR, NTL>(a, gauge, in_blk, on, p, i,
                                               z == 0 ? i + span : i - st, z == 0, acc);
        }
        {
            const int st = g.Lxh * g.L[1] * g.L[2];
            const int span = (g.L[3] - 1) * st;
            hop_dir<ST, NCL, 3, SF, true, NR, NTL>(a, gauge, in_blk, on, p, i,
                                              t == g.L[3] - 1 ? i - span : i + st,
                                              t == g.L[3] - 1, acc);
            hop_dir<ST, NCL, 3, SB, false, NR, NTL>(a, gauge, in_blk, on, p, i,
                                               t == 0 ? i + span : i - st, t == 0, acc);
        }

#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (NR > 1 && !on[r]) continue;
            cpx<R> o[12];
            cpx<R> xv[12];
            if (a.twist) {
                // diagonal twist (1 + i t g5) on the hopping term; g5 =
                // diag(1, 1, -1, -1) on the spins of the chiral basis
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const R t = k < 6 ? a.ta : -a.ta;
                    acc[r][k] = acc[r][k] + t * ci(acc[r][k]);
                }
            }
            if constexpr (XPAY) {
                load_spinor<ST, NTL, use_o32<ST, NR>()>(static_cast<const char *>(a.xs[p]) + fo[r],
                                                        g.S, i, xv);
                if (a.twist) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        const R t = k < 6 ? a.tx : -a.tx;
                        o[k] = a.sx * (xv[k] + t * ci(xv[k])) + c[r] * acc[r][k];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 12; ++k) o[k] = xv[k] + c[r] * acc[r][k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) o[k] = c[r] * acc[r][k];
            }
            if constexpr (RED != kRedCgXR)
                store_spinor<ST, WL_NT_STORE != 0>(static_cast<char *>(a.out[p]) + fo[r], g.S, i,
                                                   o);

            double *sm = sums[r];
            if constexpr (RED == kRedNorm) {
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    sm[0] += double(o[k].re) * double(o[k].re) + double(o[k].im) * double(o[k].im);
            } else if constexpr (RED == kRedDotAux) {   // <aux, out>
                cpx<R> w[12];
                load_spinor<ST>(static_cast<const char *>(a.aux[p]) + fo[r], g.S, i, w);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    sm[0] += double(w[k].re) * double(o[k].re) + double(w[k].im) * double(o[k].im);
                    sm[1] += double(w[k].re) * double(o[k].im) - double(w[k].im) * double(o[k].re);
                }
            } else if constexpr (RED == kRedCgXR) {     // x += al p; r -= al q; ||r||^2
                // the arithmetic of the separate update pass, on q in registers
                static_assert(NR == 1, "the fused CG update takes one RHS per thread");
                const R al = R(rhs_reduce(a.red, rhs0, a.nb_rhs).sc->alpha);
                cpx<R> xu[12], pu[12], ru[12];
                load_spinor<ST>(static_cast<const char *>(a.cgv[0]) + fo[r], g.S, i, xu);
                load_spinor<ST>(static_cast<const char *>(a.cgv[1]) + fo[r], g.S, i, pu);
                load_spinor<ST>(static_cast<const char *>(a.cgv[2]) + fo[r], g.S, i, ru);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    xu[k] = xu[k] + al * pu[k];
                    ru[k] = ru[k] - al * o[k];
                }
                store_spinor<ST>(static_cast<char *>(a.cgv[0]) + fo[r], g.S, i, xu);
                store_spinor<ST>(static_cast<char *>(a.cgv[2]) + fo[r], g.S, i, ru);
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    sm[0] += double(ru[k].re) * double(ru[k].re) +
                             double(ru[k].im) * double(ru[k].im);
            } else if constexpr (RED == kRedTS) {       // <out, xs>, ||out||^2
                static_assert(XPAY, "kRedTS needs the xpay source");
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    sm[0] += double(o[k].re) * double(xv[k].re) + double(o[k].im) * double(xv[k].im);
                    sm[1] += double(o[k].re) * double(xv[k].im) - double(o[k].im) * double(xv[k].re);
                    sm[2] += double(o[k].re) * double(o[k].re) + double(o[k].im) * double(o[k].im);
                }
            }
        }
    }
    if constexpr (RED != kRedNone) {
        if constexpr (NR == 1)
            block_partial<NS>(sums[0], rhs_reduce(a.red, rhs0, a.nb_rhs).partials, slot, a.nb_rhs);
        else
            block_partial_rhs<NS, NR>(sums, on, a.red, rhs0, slot, a.nb_rhs);
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <typename ST, int NCL, bool DAG, bool XPAY, int RED, int NR>
static hipError_t launch_kernel(HopArgs<Real<ST>> a, int chunk, int tgroup, hipStream_t s) {
    a.ngroups = (a.nrhs + NR - 1) / NR;
    a.nblocks = a.nb_rhs * a.ngroups;
    a.chunk = std::max(1, std::min(chunk, a.nb_rhs));
    a.tgroup = tgroup;
    // links of a one-parity launch of one RHS group are read once: streaming
    // loads keep L2 for the neighbour spinors. When both parities, or several
    // RHS groups, read every link, the later reads want it cached.
    if (a.npar == 1 && a.ngroups == 1 && WL_NT_LINKS)
        hipLaunchKernelGGL((hop_kernel<ST, NCL, DAG, XPAY, RED, NR, true>), dim3(a.nblocks),
                           dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((hop_kernel<ST, NCL, DAG, XPAY, RED, NR, false>), dim3(a.nblocks),
                           dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// RHS per thread the kernels are built for (register blocking of batches):
// FP64 and FP32 storage, no reduction or a norm; FP16 storage and the
// BiCGStab reductions use one.
template <typename ST, int RED>
constexpr bool blocked_ok() {
    return !std::is_same<ST, Half>::value && (RED == kRedNone || RED == kRedNorm);
}

// A launch shape: RHS per thread, site blocks per chunk (batches), slice
// tiles per time walk (0: lexicographic order).
struct Shape {
    int nr = 1, chunk = 1, tg = 0;
};

template <typename ST, int NCL, bool DAG, bool XPAY, int RED>
static hipError_t launch_nr(const HopArgs<Real<ST>> &a, Shape sh, hipStream_t s) {
    // with a per-RHS gauge table a thread's links are those of its first RHS,
    // so it may own only that one
    if (a.gtab) sh.nr = 1;
    if constexpr (blocked_ok<ST, RED>()) {
        switch (sh.nr) {
        case 2: return launch_kernel<ST, NCL, DAG, XPAY, RED, 2>(a, sh.chunk, sh.tg, s);
        case 3: return launch_kernel<ST, NCL, DAG, XPAY, RED, 3>(a, sh.chunk, sh.tg, s);
        case 4: return launch_kernel<ST, NCL, DAG, XPAY, RED, 4>(a, sh.chunk, sh.tg, s);
        default: break;
        }
    }
    return launch_kernel<ST, NCL, DAG, XPAY, RED, 1>(a, sh.chunk, sh.tg, s);
}

// ---- autotuning of batched launch shapes -----------------------------------
// The first launch of each shape key (precision, links, operator,
// reduction, batch size, lattice) times candidate launch shapes on the call's
// own buffers, when that is safe (no graph capture under way, the output
// aliases no input: the kernel is then idempotent and every candidate writes
// the same bits), and keeps the fastest: first the RHS-per-thread count, then
// the tile group of the time walk, then the chunk length. Choices are cached
// per process and, with WL_TUNE_FILE set, in that file; WL_TUNE=0 disables
// tuning (fixed default shape); WL_TUNE_FORCE="nr,chunk,tg" imposes a shape
// (where it applies) on every launch.
// ---- autotuner interface (state and record in wl_dslash.hip) ---------------
inline constexpr int kChunks[] = {1, 4, 16, 64, 1 << 30};
inline constexpr int kTileGroups[] = {1, 2, 4, 8, 16, 32};

struct TuneEntry {
    Shape best;
    std::vector<std::pair<Shape, float>> tried;   // candidate and its average time in us
};

std::string tune_key(const Geom &g, int prec, bool link12, bool dag, bool xpay, int red,
                     int nrhs, int npar, bool own_gauges);
bool tune_find(const std::string &key, Shape *best);
void tune_store(const std::string &key, const TuneEntry &e);
bool tuning_enabled();

// one launcher per storage precision (wl_hop_f64.hip, wl_hop_f32.hip, wl_hop_f16.hip)
hipError_t launch_storage_f64(const Geom &g, int prec, bool link12, const Phases &ph,
                              const HopCall &call, int red, hipStream_t s);
hipError_t launch_storage_f32(const Geom &g, int prec, bool link12, const Phases &ph,
                              const HopCall &call, int red, hipStream_t s);
hipError_t launch_storage_f16(const Geom &g, int prec, bool link12, const Phases &ph,
                              const HopCall &call, int red, hipStream_t s);

template <typename ST, int NCL, bool DAG, bool XPAY, int RED>
static hipError_t launch_tuned(const HopArgs<Real<ST>> &a, int prec, bool link12, hipStream_t s) {
    const bool can_nr = blocked_ok<ST, RED>() && a.nrhs >= 2 && !a.gtab;
    const bool can_tg = a.ntile_t > 1;
    Shape def;
    if (can_nr && std::is_same<ST, double>::value) def.nr = 2;
    if (const char *f = std::getenv("WL_TUNE_FORCE")) {   // fixed shape (testing)
        Shape sh;
        if (std::sscanf(f, "%d,%d,%d", &sh.nr, &sh.chunk, &sh.tg) == 3) {
            sh.nr = can_nr ? std::max(1, std::min(sh.nr, kMaxNr)) : 1;
            sh.chunk = std::max(1, sh.chunk);
            if (sh.tg < 0 || sh.tg >= a.ntile_t) sh.tg = 0;
            return launch_nr<ST, NCL, DAG, XPAY, RED>(a, sh, s);
        }
    }
    if (!can_nr && !can_tg) return launch_nr<ST, NCL, DAG, XPAY, RED>(a, def, s);
    const std::string key = tune_key(a.g, prec, link12, DAG, XPAY, RED, a.nrhs, a.npar,
                                     a.gtab != nullptr);
    {
        // a recorded shape (this process or WL_TUNE_FILE) is clamped to what
        // this launch allows: with a per-RHS gauge table every thread must own
        // one RHS, since the kernel reads the links of its first RHS only
        Shape cached;
        if (tune_find(key, &cached)) {
            if (!can_nr) cached.nr = 1;
            if (cached.tg < 0 || cached.tg >= a.ntile_t) cached.tg = 0;
            return launch_nr<ST, NCL, DAG, XPAY, RED>(a, cached, s);
        }
    }
    // is it safe to time the candidates on this call?
    bool safe = tuning_enabled();
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (safe && (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone))
        safe = false;
    for (int q = 0; q < a.npar && safe; ++q) {
        const int po = a.first_par ^ q;
        const void *o = a.out[po];
        if (o == a.in[0] || o == a.in[1] || o == a.xs[po] || o == a.aux[po] || o == a.cgv[0] ||
            o == a.cgv[1] || o == a.cgv[2])
            safe = false;
    }
    if (!safe) return launch_nr<ST, NCL, DAG, XPAY, RED>(a, def, s);

    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    TuneEntry ent;
    ent.best = def;
    float best_t = 1e30f;
    // the fused CG update changes x and r, so its candidates are timed on the
    // plain operator (the same hops, q written to `out`); the update runs once
    constexpr int TR = RED == kRedCgXR ? int(kRedNone) : RED;
    auto trial = [&](Shape sh) {
        if (err != hipSuccess) return;
        constexpr int kReps = 3;
        err = launch_nr<ST, NCL, DAG, XPAY, TR>(a, sh, s);   // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int k = 0; k < kReps && err == hipSuccess; ++k)
            err = launch_nr<ST, NCL, DAG, XPAY, TR>(a, sh, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err != hipSuccess) return;
        const float us = 1e3f * ms / kReps;
        ent.tried.push_back({sh, us});
        if (us < best_t) {
            best_t = us;
            ent.best = sh;
        }
    };
    // 1: right-hand sides per thread (lexicographic order, chunk 1)
    if (can_nr) {
        for (int nr = 1; nr <= kMaxNr && nr <= a.nrhs; ++nr) trial(Shape{nr, 1, 0});
    } else {
        trial(Shape{1, 1, 0});
    }
    // 2: slice tiles walked through time together
    if (can_tg) {
        const Shape b1 = ent.best;
        for (int tg : kTileGroups)
            if (tg < a.ntile_t) trial(Shape{b1.nr, 1, tg});
    }
    // 3: chunks of the RHS-group order
    {
        const Shape b2 = ent.best;
        const int ngroups = (a.nrhs + b2.nr - 1) / b2.nr;
        if (ngroups >= 2)
            for (int c : kChunks) {
                if (c == 1) continue;
                if (c >= a.nb_rhs && c != kChunks[sizeof kChunks / sizeof kChunks[0] - 1]) continue;
                trial(Shape{b2.nr, c, b2.tg});
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (err != hipSuccess) return err;
    tune_store(key, ent);
    // leave the chosen shape's result in place
    return launch_nr<ST, NCL, DAG, XPAY, RED>(a, ent.best, s);
}

template <typename ST, int NCL, bool DAG, bool XPAY, int RED>
static hipError_t launch_t(const HopArgs<Real<ST>> &a, const HopCall &call, int prec, bool link12,
                           hipStream_t s) {
    const hipError_t e = launch_tuned<ST, NCL, DAG, XPAY, RED>(a, prec, link12, s);
    if (e != hipSuccess || RED == kRedNone) return e;
    constexpr int NS = (RED == kRedNorm || RED == kRedCgXR) ? 1 : (RED == kRedDotAux ? 2 : 3);
    return launch_finish(a.red, NS, a.nb_rhs, a.nrhs, a.skip, s);
}

template <typename ST, int NCL, bool DAG, bool XPAY>
static hipError_t launch_red(const HopArgs<Real<ST>> &a, const HopCall &call, int prec,
                             bool link12, int red, hipStream_t s) {
    switch (red) {
    case kRedNone: return launch_t<ST, NCL, DAG, XPAY, kRedNone>(a, call, prec, link12, s);
    case kRedNorm: return launch_t<ST, NCL, DAG, XPAY, kRedNorm>(a, call, prec, link12, s);
    case kRedDotAux: return launch_t<ST, NCL, DAG, XPAY, kRedDotAux>(a, call, prec, link12, s);
    case kRedCgXR:   // the last hop of an adjoint Schur apply
        if constexpr (DAG && XPAY)
            return launch_t<ST, NCL, DAG, XPAY, kRedCgXR>(a, call, prec, link12, s);
        return hipErrorInvalidValue;
    default:
        if constexpr (XPAY) return launch_t<ST, NCL, DAG, XPAY, kRedTS>(a, call, prec, link12, s);
        return hipErrorInvalidValue;
    }
}

template <typename ST, int NCL>
static hipError_t launch_ncl(const HopArgs<Real<ST>> &a, const HopCall &call, int prec,
                             bool link12, bool dag, bool xpay, int red, hipStream_t s) {
    if (dag) {
        return xpay ? launch_red<ST, NCL, true, true>(a, call, prec, link12, red, s)
                    : launch_red<ST, NCL, true, false>(a, call, prec, link12, red, s);
    }
    return xpay ? launch_red<ST, NCL, false, true>(a, call, prec, link12, red, s)
                : launch_red<ST, NCL, false, false>(a, call, prec, link12, red, s);
}

template <typename ST>
static hipError_t launch_storage(const Geom &g, int prec, bool link12, const Phases &ph,
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
    a.ngroups = a.nrhs;
    a.chunk = 1;
    a.tgroup = 0;
    {
        const int A = g.Lxh * g.L[1] * g.L[2];
        a.ntile_t = A % kBlock == 0 ? A / kBlock : 0;
    }
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
    a.cmul = call.cmul;
    a.cpow = call.cpow;
    a.twist = call.tx != 0.0 || call.ta != 0.0 || call.sx != 1.0;
    a.tx = R(call.tx);
    a.ta = R(call.ta);
    a.sx = R(call.sx);
    a.lds = g.Lxh <= kLdsHalo;
    for (int q = 0; q < 3; ++q) a.cgv[q] = call.cg[q];
    const bool xpay = call.xs[call.first_par] != nullptr;
    return link12 ? launch_ncl<ST, 6>(a, call, prec, link12, call.dag, xpay, red, s)
                  : launch_ncl<ST, 9>(a, call, prec, link12, call.dag, xpay, red, s);
}

}  // namespace wl
