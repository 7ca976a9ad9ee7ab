// wl_blas.hip -- site-parallel vector kernels on packed spinor fields, and the
// canonical <-> packed layout and precision conversions.
//
// Every kernel maps one thread to one checkerboard site of one parity block,
// so padding entries (index >= Vh) are never touched and reductions see only
// lattice sites. Solver scalars are read from device memory (Scalars), so the
// host never waits on them inside the Krylov loop. Reductions accumulate in
// FP64 whatever the storage precision, with the deterministic last-block
// finish of wl_reduce.h.
#include "wl_internal.h"
#include "wl_reduce.h"

namespace wl {

struct BlasArgs {
    Geom g;
    int npar;
    int nblocks;          // nb_rhs * nrhs
    int nb_rhs;           // blocks per right-hand side
    int nrhs;
    size_t fstride;       // bytes between the fields of consecutive RHS
    size_t blk;           // bytes between parity blocks of one field
    char *v[6];
    double a, b;
    Scalars *sc;          // RHS r reads sc[r]
    const int *skip;
    Reduce red;
};

__device__ __forceinline__ void *blk_ptr(const BlasArgs &a, int k, int par, size_t fo) {
    return a.v[k] + fo + par * a.blk;
}

template <typename R>
__device__ __forceinline__ double norm2(const cpx<R> v[12]) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) s += double(v[k].re) * double(v[k].re) + double(v[k].im) * double(v[k].im);
    return s;
}

template <int OP> struct OpSums { static constexpr int value = 0; };
template <> struct OpSums<kOpNorm2> { static constexpr int value = 1; };
template <> struct OpSums<kOpXmy> { static constexpr int value = 1; };
template <> struct OpSums<kOpCgXR> { static constexpr int value = 1; };
template <> struct OpSums<kOpBiXR> { static constexpr int value = 3; };
template <> struct OpSums<kOpCopyNorm2> { static constexpr int value = 1; };
template <> struct OpSums<kOpCopy2Norm2> { static constexpr int value = 1; };
template <> struct OpSums<kOpNormDot> { static constexpr int value = 3; };

static int OpSumsOf(int op) { return (op == kOpBiXR || op == kOpNormDot) ? 3 : 1; }

static bool op_reduces(int op) {
    return op == kOpNorm2 || op == kOpXmy || op == kOpCgXR || op == kOpBiXR ||
           op == kOpCopyNorm2 || op == kOpCopy2Norm2 || op == kOpNormDot;
}

template <typename ST, int OP>
__global__ void __launch_bounds__(kBlock) blas_kernel(BlasArgs a) {
    using R = Real<ST>;
    constexpr int NS = OpSums<OP>::value;
    const int bl = xcd_block(blockIdx.x, a.nblocks);
    const int rhs = bl % a.nrhs;
    const int b = bl / a.nrhs;
    if (rhs_skip(a.skip, rhs)) return;
    const size_t fo = size_t(rhs) * a.fstride;
    const Scalars *sc = a.sc ? a.sc + rhs : nullptr;
    const int par = b / a.g.bpp;
    const int i = (b - par * a.g.bpp) * kBlock + threadIdx.x;
    const int S = a.g.S;
    double sums[NS > 0 ? NS : 1] = {};
    if (i < a.g.Vh) {
        cpx<R> x[12], y[12];
        if constexpr (OP == kOpZero) {
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = {R(0), R(0)};
            store_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, y);
        } else if constexpr (OP == kOpCopy || OP == kOpCopyNorm2 || OP == kOpCopy2Norm2) {
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            store_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, x);
            if constexpr (OP == kOpCopy2Norm2) store_spinor<ST>(blk_ptr(a, 2, par, fo), S, i, x);
            if constexpr (NS > 0) sums[0] = norm2(x);
        } else if constexpr (OP == kOpNorm2) {
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            sums[0] = norm2(x);
        } else if constexpr (OP == kOpRandom) {     // counter-based pseudo-random field
            // SplitMix64 finaliser of (seed, parity, site, component): the
            // value of an entry does not depend on the launch shape
            const uint64_t base = (uint64_t(a.a) << 40) ^ (uint64_t(par) << 39) ^
                                  (uint64_t(i) * 24u);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                float u[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    uint64_t z = base + uint64_t(2 * k + c) + 0x9e3779b97f4a7c15ull;
                    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
                    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
                    z ^= z >> 31;
                    u[c] = float(int64_t(z >> 11) - (int64_t(1) << 52)) * float(1.0 / 4503599627370496.0);
                }
                y[k] = {R(u[0]), R(u[1])};
            }
            store_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, y);
        } else if constexpr (OP == kOpTwist) {      // y = a (1 + i b g5) x
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            const R s = R(a.a);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const R t = R(k < 6 ? a.b : -a.b);
                y[k] = s * (x[k] + t * ci(x[k]));
            }
            store_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
        } else if constexpr (OP == kOpNormDot) {    // ||y||^2, <x, y>
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
            sums[0] = norm2(y);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                sums[1] += double(x[k].re) * double(y[k].re) + double(x[k].im) * double(y[k].im);
                sums[2] += double(x[k].re) * double(y[k].im) - double(x[k].im) * double(y[k].re);
            }
        } else if constexpr (OP == kOpXmy) {        // y = x - y
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] - y[k];
            store_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
            sums[0] = norm2(y);
        } else if constexpr (OP == kOpAxpy) {       // y += a x
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
            const R s = R(a.a);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = y[k] + s * x[k];
            store_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
        } else if constexpr (OP == kOpCgXR) {       // x += al p; r -= al q
            const R al = R(sc->alpha);
            cpx<R> p[12], q[12];
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, p);
            load_spinor<ST>(blk_ptr(a, 2, par, fo), S, i, y);
            load_spinor<ST>(blk_ptr(a, 3, par, fo), S, i, q);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = x[k] + al * p[k];
                y[k] = y[k] - al * q[k];
            }
            store_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            store_spinor<ST>(blk_ptr(a, 2, par, fo), S, i, y);
            sums[0] = norm2(y);
        } else if constexpr (OP == kOpCgP) {        // p = r + be p
            const R be = R(sc->beta);
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] + be * y[k];
            store_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
        } else if constexpr (OP == kOpBiP) {        // p = r + be (p - om v)
            const cpx<R> be{R(sc->beta_c[0]), R(sc->beta_c[1])};
            const cpx<R> om{R(sc->omega[0]), R(sc->omega[1])};
            cpx<R> v[12];
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
            load_spinor<ST>(blk_ptr(a, 2, par, fo), S, i, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] + be * (y[k] - om * v[k]);
            store_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
        } else if constexpr (OP == kOpBiS) {        // s = r - al v
            const cpx<R> al{R(sc->alpha_c[0]), R(sc->alpha_c[1])};
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] - al * y[k];
            store_spinor<ST>(blk_ptr(a, 2, par, fo), S, i, y);
        } else if constexpr (OP == kOpBiXR) {       // x += al p + om s; r = s - om t
            const cpx<R> al{R(sc->alpha_c[0]), R(sc->alpha_c[1])};
            const cpx<R> om{R(sc->omega[0]), R(sc->omega[1])};
            cpx<R> p[12], s[12], t[12];
            load_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            load_spinor<ST>(blk_ptr(a, 1, par, fo), S, i, p);
            load_spinor<ST>(blk_ptr(a, 2, par, fo), S, i, s);
            load_spinor<ST>(blk_ptr(a, 3, par, fo), S, i, t);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = x[k] + al * p[k] + om * s[k];
                y[k] = s[k] - om * t[k];
            }
            store_spinor<ST>(blk_ptr(a, 0, par, fo), S, i, x);
            store_spinor<ST>(blk_ptr(a, 4, par, fo), S, i, y);
            cpx<R> rh[12];
            load_spinor<ST>(blk_ptr(a, 5, par, fo), S, i, rh);
            sums[0] = norm2(y);
#pragma unroll
            for (int k = 0; k < 12; ++k) {   // <rhat, r>
                sums[1] += double(rh[k].re) * double(y[k].re) + double(rh[k].im) * double(y[k].im);
                sums[2] += double(rh[k].re) * double(y[k].im) - double(rh[k].im) * double(y[k].re);
            }
        }
    }
    if constexpr (NS > 0)
        block_partial<NS>(sums, rhs_reduce(a.red, rhs, a.nb_rhs).partials, b, a.nb_rhs);
}

// One block per right-hand side: add the nb partials of each sum in a fixed
// order (thread-strided, then the shuffle tree, then the waves in order),
// store the totals and run the solver epilogue.
template <int NS>
__global__ void __launch_bounds__(kBlock) finish_kernel(Reduce red, int nb, const int *skip) {
    const int r = blockIdx.x;
    if (rhs_skip(skip, r)) return;
    const Reduce rr = rhs_reduce(red, r, nb);
    double acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = 0.0;
    // kU loads in flight before they are added, in the same order as one at a
    // time (the totals keep their bits; only the load latency overlaps)
    constexpr int kU = 8;
    int b = threadIdx.x;
    for (; b + (kU - 1) * kBlock < nb; b += kU * kBlock) {
        double v[kU][NS];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int s = 0; s < NS; ++s) v[u][s] = rr.partials[s * nb + b + u * kBlock];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s] += v[u][s];
    }
    for (; b < nb; b += kBlock)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] += rr.partials[s * nb + b];
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh[kWaves][NS];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] += __shfl_xor(acc[s], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < NS; ++s) sh[wave][s] = acc[s];
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[kMaxSums] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += sh[w][s];
            tot[s] = t;
            rr.result[s] = t;
        }
        if (rr.sc) run_epilogue(rr.epilogue, tot, rr.sc);
    }
}

hipError_t launch_finish(const Reduce &red, int ns, int nb, int nrhs, const int *skip,
                         hipStream_t s) {
    const dim3 grid(nrhs), block(kBlock);
    switch (ns) {
    case 1: hipLaunchKernelGGL((finish_kernel<1>), grid, block, 0, s, red, nb, skip); break;
    case 2: hipLaunchKernelGGL((finish_kernel<2>), grid, block, 0, s, red, nb, skip); break;
    case 3: hipLaunchKernelGGL((finish_kernel<3>), grid, block, 0, s, red, nb, skip); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST>
static hipError_t blas_storage(const BlasArgs &a, int op, hipStream_t s) {
    const dim3 grid(a.nblocks), block(kBlock);
#define WL_CASE(OPV) \
    case OPV: hipLaunchKernelGGL((blas_kernel<ST, OPV>), grid, block, 0, s, a); break;
    switch (op) {
        WL_CASE(kOpZero)
        WL_CASE(kOpCopy)
        WL_CASE(kOpNorm2)
        WL_CASE(kOpXmy)
        WL_CASE(kOpCgXR)
        WL_CASE(kOpCgP)
        WL_CASE(kOpBiP)
        WL_CASE(kOpBiS)
        WL_CASE(kOpBiXR)
        WL_CASE(kOpAxpy)
        WL_CASE(kOpCopyNorm2)
        WL_CASE(kOpCopy2Norm2)
        WL_CASE(kOpNormDot)
        WL_CASE(kOpRandom)
        WL_CASE(kOpTwist)
    default: return hipErrorInvalidValue;
    }
#undef WL_CASE
    return hipGetLastError();
}

hipError_t launch_blas(const Geom &g, int prec, const BlasCall &call, hipStream_t s) {
    if (op_reduces(call.op) &&
        (!call.red || !call.red->partials || (!call.red->result && !call.red->sc)))
        return hipErrorInvalidValue;
    BlasArgs a;
    a.g = g;
    a.npar = call.npar;
    a.nrhs = call.nrhs < 1 ? 1 : call.nrhs;
    a.nb_rhs = g.bpp * call.npar;
    a.nblocks = a.nb_rhs * a.nrhs;
    a.fstride = call.fstride;
    a.blk = spinor_block_bytes(g, prec);
    for (int k = 0; k < 6; ++k) a.v[k] = static_cast<char *>(call.v[k]);
    a.a = call.a;
    a.b = call.b;
    a.sc = call.sc;
    a.skip = call.skip;
    if (call.red) a.red = *call.red;
    else a.red = Reduce{nullptr, nullptr, kEpiNone, nullptr};
    const hipError_t e =
        with_storage(prec, [&](auto tag) { return blas_storage<decltype(tag)>(a, call.op, s); });
    if (e != hipSuccess || !op_reduces(call.op)) return e;
    return launch_finish(a.red, OpSumsOf(call.op), a.nb_rhs, a.nrhs, a.skip, s);
}

// ---------------------------------------------------------------------------
// Layout conversions
// ---------------------------------------------------------------------------
struct SiteMap {
    int par, cb;
};

// canonical site s -> (parity, checkerboard index); cb = s/2 because Lx is even
__device__ __forceinline__ SiteMap site_map(const Geom &g, int s) {
    const int x = s % g.L[0];
    int r = s / g.L[0];
    const int y = r % g.L[1];
    r /= g.L[1];
    const int z = r % g.L[2];
    const int t = r / g.L[2];
    return {(x + y + z + t) & 1, s >> 1};
}

template <typename ST, int NCL>
__global__ void __launch_bounds__(kBlock) pack_gauge_kernel(Geom g, const double2 *canon,
                                                            void *packed) {
    using R = Real<ST>;
    const int gid = blockIdx.x * kBlock + threadIdx.x;   // = 4 s + mu
    if (gid >= 8 * g.Vh) return;
    const int s = gid >> 2, mu = gid & 3;
    const SiteMap m = site_map(g, s);
    cpx<R> u[9];
#pragma unroll
    for (int k = 0; k < NCL; ++k) {
        const double2 c = canon[gid * 9 + k];
        u[k] = {R(c.x), R(c.y)};
    }
    store_link_raw<ST, NCL>(packed, g.S, m.par, mu, m.cb, u);
}

// packed -> canonical link (the inverse of pack_gauge_kernel; a 12-real link
// gets its third row rebuilt as conj(row0 x row1), as the hopping kernels do)
template <typename ST, int NCL>
__global__ void __launch_bounds__(kBlock) unpack_gauge_kernel(Geom g, const void *packed,
                                                              double2 *canon) {
    using R = Real<ST>;
    const int gid = blockIdx.x * kBlock + threadIdx.x;   // = 4 s + mu
    if (gid >= 8 * g.Vh) return;
    const int s = gid >> 2, mu = gid & 3;
    const SiteMap m = site_map(g, s);
    cpx<R> u[9];
    load_link_raw<ST, NCL>(packed, g.S, m.par, mu, m.cb, u);
    if constexpr (NCL == 6) {
        u[6] = cconj(u[1] * u[5] - u[2] * u[4]);
        u[7] = cconj(u[2] * u[3] - u[0] * u[5]);
        u[8] = cconj(u[0] * u[4] - u[1] * u[3]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) canon[gid * 9 + k] = double2{double(u[k].re), double(u[k].im)};
}

template <typename ST>
__global__ void __launch_bounds__(kBlock) pack_spinor_kernel(Geom g, const double2 *canon,
                                                             void *packed, size_t blk) {
    using R = Real<ST>;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= 2 * g.Vh) return;
    const SiteMap m = site_map(g, s);
    cpx<R> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double2 c = canon[s * 12 + k];
        v[k] = {R(c.x), R(c.y)};
    }
    store_spinor<ST>(static_cast<char *>(packed) + m.par * blk, g.S, m.cb, v);
}

template <typename ST>
__global__ void __launch_bounds__(kBlock) unpack_spinor_kernel(Geom g, const void *packed,
                                                               double2 *canon, size_t blk) {
    using R = Real<ST>;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= 2 * g.Vh) return;
    const SiteMap m = site_map(g, s);
    cpx<R> v[12];
    load_spinor<ST>(static_cast<const char *>(packed) + m.par * blk, g.S, m.cb, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) canon[s * 12 + k] = double2{double(v[k].re), double(v[k].im)};
}

template <typename SS, typename SD>
__global__ void __launch_bounds__(kBlock) convert_spinor_kernel(Geom g, const char *src,
                                                                size_t sblk, char *dst,
                                                                size_t dblk) {
    const int b = blockIdx.x;
    const int par = b / g.bpp;
    const int i = (b - par * g.bpp) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cpx<Real<SS>> v[12];
    cpx<Real<SD>> w[12];
    load_spinor<SS>(src + par * sblk, g.S, i, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = {Real<SD>(v[k].re), Real<SD>(v[k].im)};
    store_spinor<SD>(dst + par * dblk, g.S, i, w);
}

template <typename SS>
__global__ void __launch_bounds__(kBlock) accum_lo_kernel(Geom g, const char *x, size_t sblk,
                                                          char *y64, size_t dblk) {
    const int b = blockIdx.x;
    const int par = b / g.bpp;
    const int i = (b - par * g.bpp) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cpx<Real<SS>> v[12];
    cpx<double> w[12];
    load_spinor<SS>(x + par * sblk, g.S, i, v);
    load_spinor<double>(y64 + par * dblk, g.S, i, w);
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = {w[k].re + double(v[k].re), w[k].im + double(v[k].im)};
    store_spinor<double>(y64 + par * dblk, g.S, i, w);
}

template <typename SD, int NCL>
__global__ void __launch_bounds__(kBlock) convert_gauge_kernel(Geom g, const void *src64,
                                                               void *dst) {
    const int b = blockIdx.x;                 // 8 * bpp blocks: (par, mu) major
    const int pm = b / g.bpp;
    const int i = (b - pm * g.bpp) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cpx<double> u[NCL];
    cpx<Real<SD>> w[NCL];
    load_link_raw<double, NCL>(src64, g.S, pm >> 2, pm & 3, i, u);
#pragma unroll
    for (int k = 0; k < NCL; ++k) w[k] = {Real<SD>(u[k].re), Real<SD>(u[k].im)};
    store_link_raw<SD, NCL>(dst, g.S, pm >> 2, pm & 3, i, w);
}

static int cdiv(long a, long b) { return int((a + b - 1) / b); }

hipError_t launch_pack_gauge(const Geom &g, int prec, bool link12, const void *canon,
                             void *packed, hipStream_t s) {
    const dim3 grid(cdiv(8L * g.Vh, kBlock)), block(kBlock);
    const double2 *c = static_cast<const double2 *>(canon);
    with_storage(prec, [&](auto tag) {
        using ST = decltype(tag);
        if (link12) hipLaunchKernelGGL((pack_gauge_kernel<ST, 6>), grid, block, 0, s, g, c, packed);
        else hipLaunchKernelGGL((pack_gauge_kernel<ST, 9>), grid, block, 0, s, g, c, packed);
        return 0;
    });
    return hipGetLastError();
}

hipError_t launch_unpack_gauge(const Geom &g, int prec, bool link12, const void *packed,
                               void *canon, hipStream_t s) {
    const dim3 grid(cdiv(8L * g.Vh, kBlock)), block(kBlock);
    double2 *c = static_cast<double2 *>(canon);
    with_storage(prec, [&](auto tag) {
        using ST = decltype(tag);
        if (link12) hipLaunchKernelGGL((unpack_gauge_kernel<ST, 6>), grid, block, 0, s, g, packed, c);
        else hipLaunchKernelGGL((unpack_gauge_kernel<ST, 9>), grid, block, 0, s, g, packed, c);
        return 0;
    });
    return hipGetLastError();
}

hipError_t launch_pack_spinor(const Geom &g, int prec, const void *canon, void *packed,
                              hipStream_t s) {
    const dim3 grid(cdiv(2L * g.Vh, kBlock)), block(kBlock);
    const double2 *c = static_cast<const double2 *>(canon);
    const size_t blk = spinor_block_bytes(g, prec);
    with_storage(prec, [&](auto tag) {
        hipLaunchKernelGGL((pack_spinor_kernel<decltype(tag)>), grid, block, 0, s, g, c, packed,
                           blk);
        return 0;
    });
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geom &g, int prec, const void *packed, void *canon,
                                hipStream_t s) {
    const dim3 grid(cdiv(2L * g.Vh, kBlock)), block(kBlock);
    double2 *c = static_cast<double2 *>(canon);
    const size_t blk = spinor_block_bytes(g, prec);
    with_storage(prec, [&](auto tag) {
        hipLaunchKernelGGL((unpack_spinor_kernel<decltype(tag)>), grid, block, 0, s, g, packed, c,
                           blk);
        return 0;
    });
    return hipGetLastError();
}

hipError_t launch_convert_spinor(const Geom &g, int npar, int src_prec, const void *src,
                                 int dst_prec, void *dst, hipStream_t s) {
    const dim3 grid(g.bpp * npar), block(kBlock);
    const char *sp = static_cast<const char *>(src);
    char *dp = static_cast<char *>(dst);
    const size_t sb = spinor_block_bytes(g, src_prec), db = spinor_block_bytes(g, dst_prec);
    with_storage(src_prec, [&](auto stag) {
        return with_storage(dst_prec, [&](auto dtag) {
            hipLaunchKernelGGL((convert_spinor_kernel<decltype(stag), decltype(dtag)>), grid, block,
                               0, s, g, sp, sb, dp, db);
            return 0;
        });
    });
    return hipGetLastError();
}

hipError_t launch_accum_lo(const Geom &g, int npar, int src_prec, const void *x, void *y64,
                           hipStream_t s) {
    const dim3 grid(g.bpp * npar), block(kBlock);
    const char *xp = static_cast<const char *>(x);
    char *yp = static_cast<char *>(y64);
    const size_t sb = spinor_block_bytes(g, src_prec), db = spinor_block_bytes(g, WL_F64);
    with_storage(src_prec, [&](auto tag) {
        hipLaunchKernelGGL((accum_lo_kernel<decltype(tag)>), grid, block, 0, s, g, xp, sb, yp, db);
        return 0;
    });
    return hipGetLastError();
}

hipError_t launch_convert_gauge(const Geom &g, bool link12, const void *src64, int dst_prec,
                                void *dst, hipStream_t s) {
    const dim3 grid(g.bpp * 8), block(kBlock);
    with_storage(dst_prec, [&](auto tag) {
        using SD = decltype(tag);
        if (link12) hipLaunchKernelGGL((convert_gauge_kernel<SD, 6>), grid, block, 0, s, g, src64, dst);
        else hipLaunchKernelGGL((convert_gauge_kernel<SD, 9>), grid, block, 0, s, g, src64, dst);
        return 0;
    });
    return hipGetLastError();
}

__global__ void set_target_kernel(Scalars *sc, double target) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->target = target;
        sc->done = 0;
        sc->status = WL_OK;
        sc->iter = 0;
    }
}

hipError_t launch_set_target(Scalars *sc, double target, hipStream_t s) {
    hipLaunchKernelGGL(set_target_kernel, dim3(1), dim3(64), 0, s, sc, target);
    return hipGetLastError();
}

struct Targets {
    double t[kMaxBatch];
};

__global__ void set_targets_kernel(Scalars *sc, Targets tg, int n) {
    const int r = threadIdx.x;
    if (blockIdx.x == 0 && r < n) {
        sc[r].target = tg.t[r];
        sc[r].done = 0;
        sc[r].status = WL_OK;
        sc[r].iter = 0;
    }
}

hipError_t launch_set_targets(Scalars *sc, const double *targets, int n, hipStream_t s) {
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    Targets tg{};
    for (int r = 0; r < n; ++r) tg.t[r] = targets[r];
    hipLaunchKernelGGL(set_targets_kernel, dim3(1), dim3(kMaxBatch), 0, s, sc, tg, n);
    return hipGetLastError();
}

__global__ void set_kappas_kernel(Scalars *sc, Targets k, int n) {
    const int r = threadIdx.x;
    if (blockIdx.x == 0 && r < n) sc[r].kappa = k.t[r];
}

hipError_t launch_set_kappas(Scalars *sc, const double *kappas, int n, hipStream_t s) {
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    Targets k{};
    for (int r = 0; r < n; ++r) k.t[r] = kappas[r];
    hipLaunchKernelGGL(set_kappas_kernel, dim3(1), dim3(kMaxBatch), 0, s, sc, k, n);
    return hipGetLastError();
}

__global__ void beta_ratio_kernel(Scalars *sc, double rr_old) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->beta = sc->rr / rr_old;
}

hipError_t launch_beta_ratio(Scalars *sc, double rr_old, hipStream_t s) {
    hipLaunchKernelGGL(beta_ratio_kernel, dim3(1), dim3(64), 0, s, sc, rr_old);
    return hipGetLastError();
}

__global__ void stop_rhs_kernel(Scalars *sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->done = 1;
}

hipError_t launch_stop_rhs(Scalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(stop_rhs_kernel, dim3(1), dim3(64), 0, s, sc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming copy: the achievable-bandwidth reference. Each thread moves
// kCopyVec 16-byte vectors, loads first, then non-temporal stores.
// ---------------------------------------------------------------------------
constexpr int kCopyVec = 4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kBlock) stream_copy_kernel(const u32x4 *src, u32x4 *dst,
                                                             size_t n) {
    const size_t base = (size_t(blockIdx.x) * kBlock * kCopyVec) + threadIdx.x;
    u32x4 v[kCopyVec];
#pragma unroll
    for (int k = 0; k < kCopyVec; ++k) {
        const size_t j = base + size_t(k) * kBlock;
        if (j < n) v[k] = __builtin_nontemporal_load(&src[j]);
    }
#pragma unroll
    for (int k = 0; k < kCopyVec; ++k) {
        const size_t j = base + size_t(k) * kBlock;
        if (j < n) __builtin_nontemporal_store(v[k], &dst[j]);
    }
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const size_t per = size_t(kBlock) * kCopyVec;
    const size_t blocks = (n + per - 1) / per;
    if (blocks > 0x7fffffffUL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, s,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n);
    return hipGetLastError();
}

}  // namespace wl
