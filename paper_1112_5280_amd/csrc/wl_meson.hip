// wl_meson.hip -- meson correlators of a point-source propagator (paper
// Sec. 4, Eq. 1):
//
//   C_Gamma(t) = - sum_xvec Tr( S^dag(x) g5 Gamma S(x) Gamma g5 ),  x = (xvec, t),
//
// where S(x) is the 12 x 12 spin-colour matrix whose column (spin b, colour c)
// is the solution of M x = b for the point source of that spin and colour,
// and the trace runs over spin and colour. t is counted from the source's
// time slice t0. The 16 Gamma_n = g_x^n0 g_y^n1 g_z^n2 g_t^n3 (bits of n) of
// the chiral basis are monomial matrices (one entry per row, in {+-1, +-i}),
// so with A = g5 Gamma and B = Gamma g5
//
//   Tr(S^dag A S B) = sum_{c, b} B[b][pB(b)] sum_{s, a} A[s][pA(s)]
//                     conj(S[(s,a),(pB(b),c)]) S[(pA(s),a),(b,c)],
//
// for every source colour c the four source-spin columns of the site suffice.
// One thread per site of a time slice; each block sums its sites' 16 values
// (shuffle tree, then its waves in order) into one partial per (Gamma, t,
// block); a second kernel adds each (Gamma, t)'s partials in block order, so
// the result does not depend on timing.
#include "wl_internal.h"
#include "wl_reduce.h"

namespace wl {

// A monomial 4 x 4 matrix: row r has its one nonzero entry i^ph[r] in column
// col[r].
struct Mono {
    int col[4];
    int ph[4];
};

constexpr Mono mono_mul(const Mono &x, const Mono &y) {
    Mono z{};
    for (int r = 0; r < 4; ++r) {
        z.col[r] = y.col[x.col[r]];
        z.ph[r] = (x.ph[r] + y.ph[x.col[r]]) & 3;
    }
    return z;
}

// The chiral basis as monomials (phases as powers of i):
//   g_k = [[0, -i sigma_k], [i sigma_k, 0]], g_t = [[0, 1], [1, 0]],
//   g5 = g_x g_y g_z g_t = diag(1, 1, -1, -1).
constexpr Mono kGamma[4] = {
    {{3, 2, 1, 0}, {3, 3, 1, 1}},   // g_x: -i, -i, i, i
    {{3, 2, 1, 0}, {2, 0, 0, 2}},   // g_y: -1, 1, 1, -1
    {{2, 3, 0, 1}, {3, 1, 1, 3}},   // g_z: -i, i, i, -i
    {{2, 3, 0, 1}, {0, 0, 0, 0}},   // g_t: 1, 1, 1, 1
};
constexpr Mono kOne{{0, 1, 2, 3}, {0, 0, 0, 0}};
constexpr Mono kG5{{0, 1, 2, 3}, {0, 0, 2, 2}};

// A_n = g5 Gamma_n and B_n = Gamma_n g5 for Gamma_n = g_x^n0 g_y^n1 g_z^n2 g_t^n3
struct MesonTab {
    Mono a[16], b[16];
};

constexpr MesonTab meson_table() {
    MesonTab t{};
    for (int n = 0; n < 16; ++n) {
        Mono g = kOne;
        for (int mu = 0; mu < 4; ++mu)
            if (n >> mu & 1) g = mono_mul(g, kGamma[mu]);
        t.a[n] = mono_mul(kG5, g);
        t.b[n] = mono_mul(g, kG5);
    }
    return t;
}

constexpr MesonTab kMeson = meson_table();

// i^k z
__device__ __forceinline__ cpx<double> ipow(int k, cpx<double> z) {
    return k == 0 ? z : k == 1 ? ci(z) : k == 2 ? cpx<double>{-z.re, -z.im}
                                                 : cpx<double>{z.im, -z.re};
}

struct MesonArgs {
    Geom g;
    const char *props;   // 12 packed FP64 full spinors, fstride bytes apart
    size_t fstride;
    size_t blk;          // bytes per parity block
    int slice;           // sites per time slice (Lx Ly Lz)
    int nchunk;          // blocks per time slice
    double2 *partials;   // [16][Lt][nchunk]
};

__global__ void __launch_bounds__(kBlock) meson_kernel(MesonArgs a) {
    const int chunk = blockIdx.x, t = blockIdx.y;
    const int xs = chunk * kBlock + threadIdx.x;
    double re[16], im[16];
#pragma unroll
    for (int n = 0; n < 16; ++n) re[n] = im[n] = 0.0;
    if (xs < a.slice) {
        const int s = xs + a.slice * t;          // canonical site index
        const int x = s % a.g.L[0];
        int r = s / a.g.L[0];
        const int y = r % a.g.L[1];
        r /= a.g.L[1];
        const int z = r % a.g.L[2];
        const int par = (x + y + z + t) & 1;
        const int i = s >> 1;                    // checkerboard index (Lx even)
        // for each source colour c and sink colour e: F[b][sp] = S[(sp, e), (b, c)]
#pragma unroll 1
        for (int c = 0; c < 3; ++c)
#pragma unroll 1
            for (int e = 0; e < 3; ++e) {
                cpx<double> F[4][4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double2 *f = reinterpret_cast<const double2 *>(
                        a.props + size_t(3 * b + c) * a.fstride + par * a.blk);
#pragma unroll
                    for (int sp = 0; sp < 4; ++sp) {
                        const double2 v = f[size_t(3 * sp + e) * a.g.S + i];
                        F[b][sp] = {v.x, v.y};
                    }
                }
                // Tr(S^dag A S B) restricted to these colours:
                //   sum_b B[b] sum_sp A[sp] conj(F[pB(b)][sp]) F[b][pA(sp)]
#pragma unroll
                for (int n = 0; n < 16; ++n) {
                    cpx<double> tn{0.0, 0.0};
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        cpx<double> u{0.0, 0.0};
#pragma unroll
                        for (int sp = 0; sp < 4; ++sp)
                            u = u + ipow(kMeson.a[n].ph[sp],
                                         cmulc(F[kMeson.b[n].col[b]][sp], F[b][kMeson.a[n].col[sp]]));
                        tn = tn + ipow(kMeson.b[n].ph[b], u);
                    }
                    re[n] -= tn.re;
                    im[n] -= tn.im;
                }
            }
    }
    // block sums: shuffle tree, then the waves in order
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh[kWaves][32];
#pragma unroll
    for (int n = 0; n < 16; ++n)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            re[n] += __shfl_xor(re[n], off, 64);
            im[n] += __shfl_xor(im[n], off, 64);
        }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int n = 0; n < 16; ++n) {
            sh[wave][2 * n] = re[n];
            sh[wave][2 * n + 1] = im[n];
        }
    __syncthreads();
    if (threadIdx.x < 16) {
        const int n = threadIdx.x;
        double sr = 0.0, si = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            sr += sh[w][2 * n];
            si += sh[w][2 * n + 1];
        }
        a.partials[(size_t(n) * a.g.L[3] + t) * a.nchunk + chunk] = double2{sr, si};
    }
}

// one thread per (Gamma, t): the slice's partials in block order
__global__ void meson_finish(const double2 *partials, int Lt, int nchunk, int t0, double *corr) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 16 * Lt) return;
    const int n = k / Lt, t = k % Lt;
    double sr = 0.0, si = 0.0;
    const double2 *p = partials + size_t(k) * nchunk;
    for (int c = 0; c < nchunk; ++c) {
        sr += p[c].x;
        si += p[c].y;
    }
    const int tr = ((t - t0) % Lt + Lt) % Lt;
    corr[2 * (n * Lt + tr)] = sr;
    corr[2 * (n * Lt + tr) + 1] = si;
}

size_t meson_workspace_bytes(const Geom &g) {
    const int slice = g.L[0] * g.L[1] * g.L[2];
    const int nchunk = (slice + kBlock - 1) / kBlock;
    return sizeof(double2) * 16 * size_t(g.L[3]) * nchunk;
}

hipError_t launch_meson(const Geom &g, const void *props, int t0, double *corr, void *work,
                        hipStream_t s) {
    MesonArgs a;
    a.g = g;
    a.props = static_cast<const char *>(props);
    a.blk = spinor_block_bytes(g, WL_F64);
    a.fstride = 2 * a.blk;
    a.slice = g.L[0] * g.L[1] * g.L[2];
    a.nchunk = (a.slice + kBlock - 1) / kBlock;
    a.partials = static_cast<double2 *>(work);
    hipLaunchKernelGGL(meson_kernel, dim3(a.nchunk, g.L[3]), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = 16 * g.L[3];
    hipLaunchKernelGGL(meson_finish, dim3((n + 255) / 256), dim3(256), 0, s, a.partials, g.L[3],
                       a.nchunk, t0, corr);
    return hipGetLastError();
}

}  // namespace wl
