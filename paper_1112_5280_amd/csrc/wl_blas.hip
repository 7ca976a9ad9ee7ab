// wl_blas.hip -- site-parallel vector kernels on packed spinor fields, and the
// canonical <-> packed layout conversions.
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
    int nblocks;
    size_t blk;           // bytes between parity blocks of one field
    char *v[6];
    double a;
    Scalars *sc;
    const int *skip;
    Reduce red;
};

template <typename R>
__device__ __forceinline__ void *blk_ptr(const BlasArgs &a, int k, int par) {
    return a.v[k] + par * a.blk;
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

template <typename R, int OP>
__global__ void __launch_bounds__(kBlock) blas_kernel(BlasArgs a) {
    if (a.skip && *a.skip) return;
    constexpr int NS = OpSums<OP>::value;
    const int b = xcd_block(blockIdx.x, a.nblocks);
    const int par = b / a.g.bpp;
    const int i = (b - par * a.g.bpp) * kBlock + threadIdx.x;
    const int S = a.g.S;
    double sums[NS > 0 ? NS : 1] = {};
    if (i < a.g.Vh) {
        cpx<R> x[12], y[12];
        if constexpr (OP == kOpZero) {
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = {R(0), R(0)};
            store_spinor<R>(blk_ptr<R>(a, 0, par), S, i, y);
        } else if constexpr (OP == kOpCopy || OP == kOpCopyNorm2 || OP == kOpCopy2Norm2) {
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            store_spinor<R>(blk_ptr<R>(a, 1, par), S, i, x);
            if constexpr (OP == kOpCopy2Norm2) store_spinor<R>(blk_ptr<R>(a, 2, par), S, i, x);
            if constexpr (NS > 0) sums[0] = norm2(x);
        } else if constexpr (OP == kOpNorm2) {
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            sums[0] = norm2(x);
        } else if constexpr (OP == kOpXmy) {        // y = x - y
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            load_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] - y[k];
            store_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
            sums[0] = norm2(y);
        } else if constexpr (OP == kOpAxpy) {       // y += a x
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            load_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
            const R s = R(a.a);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = y[k] + s * x[k];
            store_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
        } else if constexpr (OP == kOpCgXR) {       // x += al p; r -= al q
            const R al = R(a.sc->alpha);
            cpx<R> p[12], q[12];
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            load_spinor<R>(blk_ptr<R>(a, 1, par), S, i, p);
            load_spinor<R>(blk_ptr<R>(a, 2, par), S, i, y);
            load_spinor<R>(blk_ptr<R>(a, 3, par), S, i, q);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = x[k] + al * p[k];
                y[k] = y[k] - al * q[k];
            }
            store_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            store_spinor<R>(blk_ptr<R>(a, 2, par), S, i, y);
            sums[0] = norm2(y);
        } else if constexpr (OP == kOpCgP) {        // p = r + be p
            const R be = R(a.sc->beta);
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            load_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] + be * y[k];
            store_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
        } else if constexpr (OP == kOpBiP) {        // p = r + be (p - om v)
            const cpx<R> be{R(a.sc->beta_c[0]), R(a.sc->beta_c[1])};
            const cpx<R> om{R(a.sc->omega[0]), R(a.sc->omega[1])};
            cpx<R> v[12];
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            load_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
            load_spinor<R>(blk_ptr<R>(a, 2, par), S, i, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] + be * (y[k] - om * v[k]);
            store_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
        } else if constexpr (OP == kOpBiS) {        // s = r - al v
            const cpx<R> al{R(a.sc->alpha_c[0]), R(a.sc->alpha_c[1])};
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            load_spinor<R>(blk_ptr<R>(a, 1, par), S, i, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = x[k] - al * y[k];
            store_spinor<R>(blk_ptr<R>(a, 2, par), S, i, y);
        } else if constexpr (OP == kOpBiXR) {       // x += al p + om s; r = s - om t
            const cpx<R> al{R(a.sc->alpha_c[0]), R(a.sc->alpha_c[1])};
            const cpx<R> om{R(a.sc->omega[0]), R(a.sc->omega[1])};
            cpx<R> p[12], s[12], t[12];
            load_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            load_spinor<R>(blk_ptr<R>(a, 1, par), S, i, p);
            load_spinor<R>(blk_ptr<R>(a, 2, par), S, i, s);
            load_spinor<R>(blk_ptr<R>(a, 3, par), S, i, t);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = x[k] + al * p[k] + om * s[k];
                y[k] = s[k] - om * t[k];
            }
            store_spinor<R>(blk_ptr<R>(a, 0, par), S, i, x);
            store_spinor<R>(blk_ptr<R>(a, 4, par), S, i, y);
            cpx<R> rh[12];
            load_spinor<R>(blk_ptr<R>(a, 5, par), S, i, rh);
            sums[0] = norm2(y);
#pragma unroll
            for (int k = 0; k < 12; ++k) {   // <rhat, r>
                sums[1] += double(rh[k].re) * double(y[k].re) + double(rh[k].im) * double(y[k].im);
                sums[2] += double(rh[k].re) * double(y[k].im) - double(rh[k].im) * double(y[k].re);
            }
        }
    }
    if constexpr (NS > 0) grid_reduce<NS>(sums, a.red, b, a.nblocks);
}

template <typename R>
static hipError_t blas_prec(const BlasArgs &a, int op, hipStream_t s) {
    const dim3 grid(a.nblocks), block(kBlock);
#define WL_CASE(OPV) \
    case OPV: hipLaunchKernelGGL((blas_kernel<R, OPV>), grid, block, 0, s, a); break;
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
    default: return hipErrorInvalidValue;
    }
#undef WL_CASE
    return hipGetLastError();
}

hipError_t launch_blas(const Geom &g, int prec, const BlasCall &call, hipStream_t s) {
    const bool reduces = call.op == kOpNorm2 || call.op == kOpXmy || call.op == kOpCgXR ||
                         call.op == kOpBiXR || call.op == kOpCopyNorm2 || call.op == kOpCopy2Norm2;
    if (reduces && (!call.red || !call.red->partials || !call.red->counter || !call.red->result))
        return hipErrorInvalidValue;
    BlasArgs a;
    a.g = g;
    a.npar = call.npar;
    a.nblocks = g.bpp * call.npar;
    a.blk = spinor_block_bytes(g, prec);
    for (int k = 0; k < 6; ++k) a.v[k] = static_cast<char *>(call.v[k]);
    a.a = call.a;
    a.sc = call.sc;
    a.skip = call.skip;
    if (call.red) a.red = *call.red;
    else a.red = Reduce{nullptr, nullptr, nullptr, kEpiNone, nullptr};
    return prec == WL_F64 ? blas_prec<double>(a, call.op, s) : blas_prec<float>(a, call.op, s);
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

template <typename R, int NCL>
__global__ void __launch_bounds__(kBlock) pack_gauge_kernel(Geom g, const double2 *canon,
                                                            void *packed) {
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
    using F = LinkFmt<R, NCL>;
    typename F::T *base = static_cast<typename F::T *>(packed) + (m.par * 4 + mu) * F::NCH * g.S;
    store_cplx<R, NCL, F::CW>(base, g.S, m.cb, u);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) pack_spinor_kernel(Geom g, const double2 *canon,
                                                             void *packed, size_t blk) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= 2 * g.Vh) return;
    const SiteMap m = site_map(g, s);
    cpx<R> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double2 c = canon[s * 12 + k];
        v[k] = {R(c.x), R(c.y)};
    }
    store_spinor<R>(static_cast<char *>(packed) + m.par * blk, g.S, m.cb, v);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) unpack_spinor_kernel(Geom g, const void *packed,
                                                               double2 *canon, size_t blk) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= 2 * g.Vh) return;
    const SiteMap m = site_map(g, s);
    cpx<R> v[12];
    load_spinor<R>(static_cast<const char *>(packed) + m.par * blk, g.S, m.cb, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) canon[s * 12 + k] = double2{double(v[k].re), double(v[k].im)};
}

template <typename RS, typename RD>
__global__ void __launch_bounds__(kBlock) convert_spinor_kernel(Geom g, const char *src,
                                                                size_t sblk, char *dst,
                                                                size_t dblk) {
    const int b = blockIdx.x;
    const int par = b / g.bpp;
    const int i = (b - par * g.bpp) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cpx<RS> v[12];
    cpx<RD> w[12];
    load_spinor<RS>(src + par * sblk, g.S, i, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = {RD(v[k].re), RD(v[k].im)};
    store_spinor<RD>(dst + par * dblk, g.S, i, w);
}

__global__ void __launch_bounds__(kBlock) accum_f32_kernel(Geom g, const char *x32, size_t sblk,
                                                           char *y64, size_t dblk) {
    const int b = blockIdx.x;
    const int par = b / g.bpp;
    const int i = (b - par * g.bpp) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cpx<float> v[12];
    cpx<double> w[12];
    load_spinor<float>(x32 + par * sblk, g.S, i, v);
    load_spinor<double>(y64 + par * dblk, g.S, i, w);
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = {w[k].re + double(v[k].re), w[k].im + double(v[k].im)};
    store_spinor<double>(y64 + par * dblk, g.S, i, w);
}

template <int NCL>
__global__ void __launch_bounds__(kBlock) convert_gauge_kernel(Geom g, const void *src64,
                                                               void *dst32) {
    const int b = blockIdx.x;                 // 8 * bpp blocks: (par, mu) major
    const int pm = b / g.bpp;
    const int i = (b - pm * g.bpp) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    using F64 = LinkFmt<double, NCL>;
    using F32 = LinkFmt<float, NCL>;
    cpx<double> u[NCL];
    cpx<float> w[NCL];
    load_cplx<double, NCL, F64::CW>(static_cast<const typename F64::T *>(src64) + pm * F64::NCH * g.S,
                                    g.S, i, u);
#pragma unroll
    for (int k = 0; k < NCL; ++k) w[k] = {float(u[k].re), float(u[k].im)};
    store_cplx<float, NCL, F32::CW>(static_cast<typename F32::T *>(dst32) + pm * F32::NCH * g.S,
                                    g.S, i, w);
}

static int cdiv(long a, long b) { return int((a + b - 1) / b); }

hipError_t launch_pack_gauge(const Geom &g, int prec, bool link12, const void *canon,
                             void *packed, hipStream_t s) {
    const dim3 grid(cdiv(8L * g.Vh, kBlock)), block(kBlock);
    const double2 *c = static_cast<const double2 *>(canon);
    if (prec == WL_F64) {
        if (link12) hipLaunchKernelGGL((pack_gauge_kernel<double, 6>), grid, block, 0, s, g, c, packed);
        else hipLaunchKernelGGL((pack_gauge_kernel<double, 9>), grid, block, 0, s, g, c, packed);
    } else {
        if (link12) hipLaunchKernelGGL((pack_gauge_kernel<float, 6>), grid, block, 0, s, g, c, packed);
        else hipLaunchKernelGGL((pack_gauge_kernel<float, 9>), grid, block, 0, s, g, c, packed);
    }
    return hipGetLastError();
}

hipError_t launch_pack_spinor(const Geom &g, int prec, const void *canon, void *packed,
                              hipStream_t s) {
    const dim3 grid(cdiv(2L * g.Vh, kBlock)), block(kBlock);
    const double2 *c = static_cast<const double2 *>(canon);
    const size_t blk = spinor_block_bytes(g, prec);
    if (prec == WL_F64) hipLaunchKernelGGL((pack_spinor_kernel<double>), grid, block, 0, s, g, c, packed, blk);
    else hipLaunchKernelGGL((pack_spinor_kernel<float>), grid, block, 0, s, g, c, packed, blk);
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geom &g, int prec, const void *packed, void *canon,
                                hipStream_t s) {
    const dim3 grid(cdiv(2L * g.Vh, kBlock)), block(kBlock);
    double2 *c = static_cast<double2 *>(canon);
    const size_t blk = spinor_block_bytes(g, prec);
    if (prec == WL_F64) hipLaunchKernelGGL((unpack_spinor_kernel<double>), grid, block, 0, s, g, packed, c, blk);
    else hipLaunchKernelGGL((unpack_spinor_kernel<float>), grid, block, 0, s, g, packed, c, blk);
    return hipGetLastError();
}

hipError_t launch_convert_spinor(const Geom &g, int npar, int src_prec, const void *src,
                                 int dst_prec, void *dst, hipStream_t s) {
    const dim3 grid(g.bpp * npar), block(kBlock);
    const char *sp = static_cast<const char *>(src);
    char *dp = static_cast<char *>(dst);
    const size_t sb = spinor_block_bytes(g, src_prec), db = spinor_block_bytes(g, dst_prec);
    if (src_prec == WL_F64 && dst_prec == WL_F32)
        hipLaunchKernelGGL((convert_spinor_kernel<double, float>), grid, block, 0, s, g, sp, sb, dp, db);
    else if (src_prec == WL_F32 && dst_prec == WL_F64)
        hipLaunchKernelGGL((convert_spinor_kernel<float, double>), grid, block, 0, s, g, sp, sb, dp, db);
    else if (src_prec == WL_F64)
        hipLaunchKernelGGL((convert_spinor_kernel<double, double>), grid, block, 0, s, g, sp, sb, dp, db);
    else
        hipLaunchKernelGGL((convert_spinor_kernel<float, float>), grid, block, 0, s, g, sp, sb, dp, db);
    return hipGetLastError();
}

hipError_t launch_accum_f32(const Geom &g, int npar, const void *x32, void *y64, hipStream_t s) {
    const dim3 grid(g.bpp * npar), block(kBlock);
    hipLaunchKernelGGL(accum_f32_kernel, grid, block, 0, s, g, static_cast<const char *>(x32),
                       spinor_block_bytes(g, WL_F32), static_cast<char *>(y64),
                       spinor_block_bytes(g, WL_F64));
    return hipGetLastError();
}

hipError_t launch_convert_gauge(const Geom &g, bool link12, const void *src64, void *dst32,
                                hipStream_t s) {
    const dim3 grid(g.bpp * 8), block(kBlock);
    if (link12) hipLaunchKernelGGL((convert_gauge_kernel<6>), grid, block, 0, s, g, src64, dst32);
    else hipLaunchKernelGGL((convert_gauge_kernel<9>), grid, block, 0, s, g, src64, dst32);
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

}  // namespace wl
