// wl_reduce.h -- deterministic reductions, solver epilogues, block order.
//
// A reducing kernel leaves one partial sum per block and per summed quantity
// (block_partial); a one-block-per-RHS finish kernel then adds the partials in
// a fixed order, stores the totals and runs the solver epilogue
// (finish_reduce). No atomics are involved, so the totals are bitwise
// reproducible and nothing has to be reset between launches.
#pragma once

#include "wl_internal.h"

namespace wl {

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Updates of the solver scalars once the totals of a fused reduction are known.
// Runs on one thread of the finish kernel.
__device__ inline void run_epilogue(int epi, const double *tot, Scalars *sc) {
    switch (epi) {
    case kEpiCgInit: {
        const double rr = tot[0];
        sc->rr = rr;
        sc->iter = 0;
        sc->status = WL_OK;
        sc->alpha = 0.0;
        sc->beta = 0.0;
        if (!finite(rr)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
        } else {
            sc->done = rr <= sc->target;
        }
        break;
    }
    case kEpiCgPap: {
        const double pap = tot[0];
        sc->pap = pap;
        if (!(pap > 0.0) || !finite(pap)) {
            sc->alpha = 0.0;
            sc->done = 1;
            sc->status = (sc->rr == 0.0) ? WL_OK : WL_BREAKDOWN;
        } else {
            sc->alpha = sc->rr / pap;
        }
        break;
    }
    case kEpiCgRr: {
        const double rr = tot[0];
        sc->iter += 1;
        if (!finite(rr)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
            break;
        }
        sc->beta = rr / sc->rr;
        sc->rr = rr;
        if (rr <= sc->target) sc->done = 1;
        break;
    }
    case kEpiBiInit: {
        const double rr = tot[0];
        sc->rr = rr;
        sc->rho[0] = rr;
        sc->rho[1] = 0.0;
        sc->alpha_c[0] = 1.0;
        sc->alpha_c[1] = 0.0;
        sc->omega[0] = 1.0;
        sc->omega[1] = 0.0;
        sc->beta_c[0] = 0.0;
        sc->beta_c[1] = 0.0;
        sc->iter = 0;
        sc->status = WL_OK;
        if (!finite(rr)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
        } else {
            sc->done = rr <= sc->target;
        }
        break;
    }
    case kEpiBiAlpha: {   // alpha = rho / <rhat, v>
        const double a = tot[0], b = tot[1];
        const double d = a * a + b * b;
        if (!(d > 0.0) || !finite(d)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
            break;
        }
        const double r0 = sc->rho[0], r1 = sc->rho[1];
        sc->alpha_c[0] = (r0 * a + r1 * b) / d;
        sc->alpha_c[1] = (r1 * a - r0 * b) / d;
        break;
    }
    case kEpiBiOmega: {   // omega = <t, s> / <t, t>
        const double tt = tot[2];
        if (!finite(tt) || !finite(tot[0]) || !finite(tot[1])) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
            break;
        }
        if (tt > 0.0) {
            sc->omega[0] = tot[0] / tt;
            sc->omega[1] = tot[1] / tt;
        } else {          // t = M s = 0 means s = 0: the step with alpha alone is exact
            sc->omega[0] = 0.0;
            sc->omega[1] = 0.0;
        }
        break;
    }
    case kEpiBiRho: {     // rr = ||r||^2, rho_new = <rhat, r>
        const double rr = tot[0];
        const double n0 = tot[1], n1 = tot[2];
        sc->iter += 1;
        if (!finite(rr) || !finite(n0) || !finite(n1)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
            break;
        }
        sc->rr = rr;
        if (rr <= sc->target) {
            sc->done = 1;
            break;
        }
        // beta = (rho_new / rho) (alpha / omega)
        const double r0 = sc->rho[0], r1 = sc->rho[1];
        const double w0 = sc->omega[0], w1 = sc->omega[1];
        const double dr = r0 * r0 + r1 * r1, dw = w0 * w0 + w1 * w1;
        if (!(dr > 0.0) || !(dw > 0.0) || !(n0 * n0 + n1 * n1 > 0.0)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
            break;
        }
        const double q0 = (n0 * r0 + n1 * r1) / dr, q1 = (n1 * r0 - n0 * r1) / dr;
        const double a0 = sc->alpha_c[0], a1 = sc->alpha_c[1];
        const double s0 = (a0 * w0 + a1 * w1) / dw, s1 = (a1 * w0 - a0 * w1) / dw;
        sc->beta_c[0] = q0 * s0 - q1 * s1;
        sc->beta_c[1] = q0 * s1 + q1 * s0;
        sc->rho[0] = n0;
        sc->rho[1] = n1;
        break;
    }
    case kEpiBiInitShadow: {   // a fresh sequence whose shadow rhat is not r
        const double rr = tot[0];
        sc->rr = rr;
        sc->rho[0] = tot[1];
        sc->rho[1] = tot[2];
        sc->alpha_c[0] = 1.0;
        sc->alpha_c[1] = 0.0;
        sc->omega[0] = 1.0;
        sc->omega[1] = 0.0;
        sc->beta_c[0] = 0.0;
        sc->beta_c[1] = 0.0;
        sc->iter = 0;
        sc->status = WL_OK;
        if (!finite(rr) || !finite(tot[1]) || !finite(tot[2])) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
        } else {
            sc->done = rr <= sc->target;
        }
        break;
    }
    case kEpiBiResume: {  // the residual was replaced by a recomputed one:
        // rho_new = <rhat, r> and beta = (rho_new / rho)(alpha / omega) for the
        // direction update of the iteration whose end was the stop point
        const double rr = tot[0];
        const double n0 = tot[1], n1 = tot[2];
        if (!finite(rr) || !finite(n0) || !finite(n1)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
            break;
        }
        sc->rr = rr;
        const double r0 = sc->rho[0], r1 = sc->rho[1];
        const double w0 = sc->omega[0], w1 = sc->omega[1];
        const double dr = r0 * r0 + r1 * r1, dw = w0 * w0 + w1 * w1;
        if (!(dr > 0.0) || !(dw > 0.0) || !(n0 * n0 + n1 * n1 > 0.0)) {
            sc->done = 1;
            sc->status = WL_BREAKDOWN;
            break;
        }
        const double q0 = (n0 * r0 + n1 * r1) / dr, q1 = (n1 * r0 - n0 * r1) / dr;
        const double a0 = sc->alpha_c[0], a1 = sc->alpha_c[1];
        const double s0 = (a0 * w0 + a1 * w1) / dw, s1 = (a1 * w0 - a0 * w1) / dw;
        sc->beta_c[0] = q0 * s0 - q1 * s1;
        sc->beta_c[1] = q0 * s1 + q1 * s0;
        sc->rho[0] = n0;
        sc->rho[1] = n1;
        sc->done = rr <= sc->target;
        break;
    }
    default:
        break;
    }
}

// Sum NS per-thread values over the block (wave64 shuffle tree, then the
// waves in order) and store the block's totals at partials[s * nb + slot].
// Must be reached by every thread of the block.
template <int NS>
__device__ __forceinline__ void block_partial(double (&v)[NS], double *partials, int slot,
                                              int nb) {
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh[kWaves][NS];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int s = 0; s < NS; ++s) v[s] += __shfl_xor(v[s], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < NS; ++s) sh[wave][s] = v[s];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += sh[w][s];
            partials[s * nb + slot] = t;
        }
    }
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous run
// of logical blocks so neighbouring sites share an L2.
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int k = b & 7, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

// Batches of right-hand sides: RHS r owns the r-th Scalars entry and its own
// nb partial slots per summed quantity.
__device__ __forceinline__ Reduce rhs_reduce(const Reduce &red, int r, int nb) {
    Reduce o = red;
    o.partials = red.partials + size_t(r) * kMaxSums * nb;
    if (red.sc) {
        o.sc = red.sc + r;
        o.result = o.sc->sums;
    } else {
        o.result = red.result + r * kMaxSums;
    }
    return o;
}

// `skip` points at the `done` flag of RHS 0; RHS r's flag is one Scalars further
__device__ __forceinline__ bool rhs_skip(const int *skip, int r) {
    return skip && *reinterpret_cast<const int *>(reinterpret_cast<const char *>(skip) +
                                                  size_t(r) * sizeof(Scalars));
}

}  // namespace wl
