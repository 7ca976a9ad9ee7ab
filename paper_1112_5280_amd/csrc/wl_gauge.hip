// wl_gauge.hip -- pure-gauge kernels on the canonical complex128 gauge field
// U[V][4][3][3] (the layout wl_pack_gauge reads): the SU(3) heat bath of the
// Wilson plaquette action (paper Sec. 3: the heatbath of the pure-gauge side,
// after Creutz) and the mean plaquette.
//
// Heat bath: S = beta sum_P (1 - Re Tr U_P / 3). A sweep updates, for
// mu = 0..3, the links U_mu(x) of the even and then the odd sites (one thread
// per link; links of one direction and parity are not in each other's
// staples). Each link gets the Cabibbo-Marinari update over the SU(2)
// subgroups on rows/columns (0,1), (1,2), (0,2): with W = U A (A the staple
// sum) and w its 2 x 2 block, the SU(2) element is r = X V, V the SU(2)
// direction of b = (Re(w00 + w11), -Im(w01 + w10), Re(w10 - w01),
// -Im(w00 - w11)) / 2, and X drawn with density exp(alpha X0), alpha =
// 2 beta |b| / 3: X0 from its density sqrt(1 - X0^2) exp(alpha X0) by
// rejection (Kennedy-Pendleton candidates for alpha >= 1; below, where those
// are seldom accepted, the first coordinate of a uniform point of the unit
// disk, accepted with probability exp(alpha (X0 - 1))), the other three
// components uniform on their sphere; a zero b (V undefined) gives alpha = 0
// and V = 1. Random numbers come from Philox4x32-10 keyed by the seed,
// with counters (site, mu + 4 subgroup + 16 attempt, sweep, draw), so a link's
// update does not depend on the launch shape or on the other links' timing.
#include "wl_reduce.h"

namespace wl {

namespace {

typedef cpx<double> C;

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__device__ __forceinline__ void unif4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                      uint32_t k0, uint32_t k1, double u[4]) {
    uint32_t o[4];
    philox4x32_10(a, b, c, d, k0, k1, o);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = (double(o[i]) + 0.5) * (1.0 / 4294967296.0);
}

// rejection attempts per draw: each is accepted with probability >= 0.41, so
// a draw fails (and its subgroup keeps the link) with probability < 1e-29
constexpr int kHbTries = 128;

struct GaugeArgs {
    double2 *U;          // canonical [V][4][9] complex, or the packed FP64 field
    int L[4];
    int V;
    int mu, par;
    double beta;
    uint32_t sweep, k0, k1;
    size_t S;            // packed: sites per parity block (Vh rounded up)
};

// Link U_mu at lexicographic site s with coordinates c. Canonical: its 9
// complex numbers are contiguous. Packed (the FP64 18-real layout of
// wl_pack_gauge): entry k of the links of parity p and direction mu is an
// array of S complex numbers indexed by the checkerboard index s / 2, so
// neighbouring threads read neighbouring addresses.
template <bool PACKED>
__device__ __forceinline__ const double2 *link_at(const double2 *U, size_t S, int s,
                                                  const int c[4], int mu, size_t *stride) {
    if constexpr (PACKED) {
        const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
        *stride = S;
        return U + size_t(par * 4 + mu) * 9 * S + (s >> 1);
    } else {
        *stride = 1;
        return U + (size_t(s) * 4 + mu) * 9;
    }
}

template <bool PACKED>
__device__ __forceinline__ void ld(const double2 *U, size_t S, int s, const int c[4], int mu,
                                   C m[9]) {
    size_t st;
    const double2 *p = link_at<PACKED>(U, S, s, c, mu, &st);
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = {p[k * st].x, p[k * st].y};
}

// c = a b, a b^dag, a^dag b
__device__ __forceinline__ void mm(const C a[9], const C b[9], C c[9]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}
__device__ __forceinline__ void mmd(const C a[9], const C b[9], C c[9]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = a[3 * i] * cconj(b[3 * j]) + a[3 * i + 1] * cconj(b[3 * j + 1]) +
                           a[3 * i + 2] * cconj(b[3 * j + 2]);
}
__device__ __forceinline__ void mdm(const C a[9], const C b[9], C c[9]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = cmulc(a[i], b[j]) + cmulc(a[3 + i], b[3 + j]) + cmulc(a[6 + i], b[6 + j]);
}

__device__ __forceinline__ int site_of(const int L[4], const int c[4]) {
    return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]));
}

template <bool PACKED>
__global__ void __launch_bounds__(kBlock) heatbath_kernel(GaugeArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;   // index among the sites of parity par
    if (i >= a.V / 2) return;
    // i -> coordinates: x runs over the sites of parity par in each row
    const int lxh = a.L[0] / 2;
    int c[4];
    int r = i / lxh;
    c[1] = r % a.L[1];
    r /= a.L[1];
    c[2] = r % a.L[2];
    c[3] = r / a.L[2];
    c[0] = 2 * (i % lxh) + ((c[1] + c[2] + c[3] + a.par) & 1);
    const int s = site_of(a.L, c);
    const int mu = a.mu;
    // staple sum
    C A[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = {0.0, 0.0};
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int e[4] = {c[0], c[1], c[2], c[3]};
        e[mu] = (c[mu] + 1) % a.L[mu];
        const int xpmu = site_of(a.L, e);
        int f[4] = {c[0], c[1], c[2], c[3]};
        f[nu] = (c[nu] + 1) % a.L[nu];
        const int xpnu = site_of(a.L, f);
        int g[4] = {c[0], c[1], c[2], c[3]};
        g[nu] = (c[nu] - 1 + a.L[nu]) % a.L[nu];
        const int xmnu = site_of(a.L, g);
        int h[4] = {g[0], g[1], g[2], g[3]};
        h[mu] = (h[mu] + 1) % a.L[mu];
        const int xpmu_mnu = site_of(a.L, h);
        C m1[9], m2[9], t[9];
        ld<PACKED>(a.U, a.S, xpmu, e, nu, m1);     // U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        ld<PACKED>(a.U, a.S, xpnu, f, mu, m2);
        mmd(m1, m2, t);
        ld<PACKED>(a.U, a.S, s, c, nu, m1);
        mmd(t, m1, m2);
#pragma unroll
        for (int k = 0; k < 9; ++k) A[k] = A[k] + m2[k];
        ld<PACKED>(a.U, a.S, xmnu, g, mu, m1);     // (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu)
        ld<PACKED>(a.U, a.S, xpmu_mnu, h, nu, m2);
        mm(m1, m2, t);
        ld<PACKED>(a.U, a.S, xmnu, g, nu, m1);
        mdm(t, m1, m2);
#pragma unroll
        for (int k = 0; k < 9; ++k) A[k] = A[k] + m2[k];
    }
    C u[9];
    ld<PACKED>(a.U, a.S, s, c, mu, u);
    constexpr int sub[3][2] = {{0, 1}, {1, 2}, {0, 2}};
#pragma unroll
    for (int gidx = 0; gidx < 3; ++gidx) {
        const int ii = sub[gidx][0], jj = sub[gidx][1];
        C W[9];
        mm(u, A, W);
        const C w00 = W[4 * ii], w01 = W[3 * ii + jj], w10 = W[3 * jj + ii], w11 = W[4 * jj];
        const double b0 = 0.5 * (w00.re + w11.re), b1 = -0.5 * (w01.im + w10.im);
        const double b2 = 0.5 * (w10.re - w01.re), b3 = -0.5 * (w00.im - w11.im);
        const double k = sqrt(b0 * b0 + b1 * b1 + b2 * b2 + b3 * b3);
        const bool flat = !(k > 0.0);              // V = 1, alpha = 0
        const uint32_t tag = uint32_t(mu) | (uint32_t(gidx) << 2);
        const double alpha = flat ? 0.0 : 2.0 * a.beta * k / 3.0;
        double x0 = 2.0;
        for (int n = 0; n < kHbTries; ++n) {
            double q[4];
            unif4(uint32_t(s), tag + 16u * uint32_t(n), a.sweep, 0u, a.k0, a.k1, q);
            if (alpha < 1.0) {                     // unit disk, exp(alpha (x - 1))
                const double x = sqrt(q[0]) * cos(2.0 * M_PI * q[1]);
                if (q[2] <= exp(alpha * (x - 1.0))) {
                    x0 = x;
                    break;
                }
            } else {                               // Kennedy-Pendleton
                const double cs = cos(2.0 * M_PI * q[1]);
                const double l2 = -(log(q[0]) + cs * cs * log(q[2])) / (2.0 * alpha);
                if (q[3] * q[3] <= 1.0 - l2) {
                    x0 = 1.0 - 2.0 * l2;
                    break;
                }
            }
        }
        if (x0 > 1.0) continue;   // no acceptance: this subgroup keeps its link
        double d[4];
        unif4(uint32_t(s), tag, a.sweep, 1u, a.k0, a.k1, d);
        const double ct = 2.0 * d[0] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double ph = 2.0 * M_PI * d[1], rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
        const double x1 = rad * st * cos(ph), x2 = rad * st * sin(ph), x3 = rad * ct;
        const double v0 = flat ? 1.0 : b0 / k, v1 = flat ? 0.0 : b1 / k;
        const double v2 = flat ? 0.0 : b2 / k, v3 = flat ? 0.0 : b3 / k;
        const C X[4] = {{x0, x3}, {x2, x1}, {-x2, x1}, {x0, -x3}};
        const C Vm[4] = {{v0, v3}, {v2, v1}, {-v2, v1}, {v0, -v3}};
        const C rr[4] = {X[0] * Vm[0] + X[1] * Vm[2], X[0] * Vm[1] + X[1] * Vm[3],
                         X[2] * Vm[0] + X[3] * Vm[2], X[2] * Vm[1] + X[3] * Vm[3]};
#pragma unroll
        for (int col = 0; col < 3; ++col) {
            const C ui = u[3 * ii + col], uj = u[3 * jj + col];
            u[3 * ii + col] = rr[0] * ui + rr[1] * uj;
            u[3 * jj + col] = rr[2] * ui + rr[3] * uj;
        }
    }
    size_t st;
    double2 *p = const_cast<double2 *>(link_at<PACKED>(a.U, a.S, s, c, mu, &st));
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k * st] = double2{u[k].re, u[k].im};
}

// Sum over a block's sites of sum_{mu < nu} Re Tr U_mu nu(x) / 3; one partial per block.
// Canonical: thread n takes lexicographic site n; packed: the sites of parity
// n / Vh in checkerboard order (coalesced loads of the packed field).
template <bool PACKED>
__global__ void __launch_bounds__(kBlock) plaquette_kernel(const double2 *U, Geom g,
                                                           double *partials) {
    const int V = 2 * g.Vh;
    const int n = blockIdx.x * kBlock + threadIdx.x;
    double sum[1] = {0.0};
    if (n < V) {
        int c[4];
        if constexpr (PACKED) {
            const int par = n >= g.Vh ? 1 : 0;
            const int i = n - par * g.Vh;
            const int xh = i % g.Lxh;
            int r = i / g.Lxh;
            c[1] = r % g.L[1];
            r /= g.L[1];
            c[2] = r % g.L[2];
            c[3] = r / g.L[2];
            c[0] = 2 * xh + ((c[1] + c[2] + c[3] + par) & 1);
        } else {
            int r = n;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                c[m] = r % g.L[m];
                r /= g.L[m];
            }
        }
        const int s = site_of(g.L, c);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                int e[4] = {c[0], c[1], c[2], c[3]};
                e[mu] = (c[mu] + 1) % g.L[mu];
                int f[4] = {c[0], c[1], c[2], c[3]};
                f[nu] = (c[nu] + 1) % g.L[nu];
                C m1[9], m2[9], t[9];
                const size_t S = g.S;
                ld<PACKED>(U, S, s, c, mu, m1);   // U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                ld<PACKED>(U, S, site_of(g.L, e), e, nu, m2);
                mm(m1, m2, t);
                ld<PACKED>(U, S, site_of(g.L, f), f, mu, m1);
                mmd(t, m1, m2);
                ld<PACKED>(U, S, s, c, nu, m1);
                double tr = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        tr += m2[3 * i + k].re * m1[3 * i + k].re + m2[3 * i + k].im * m1[3 * i + k].im;
                sum[0] += tr / 3.0;
            }
    }
    block_partial<1>(sum, partials, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) plaquette_finish(const double *partials, int nb,
                                                           double norm, double *out) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += kBlock) v[0] += partials[b];
    __shared__ double tot[1];
    block_partial<1>(v, tot, 0, 1);
    __syncthreads();
    if (threadIdx.x == 0) *out = tot[0] * norm;
}

}  // namespace

hipError_t launch_heatbath_field(const Geom &g, void *field, bool packed, double beta,
                                 int nsweeps, uint32_t sweep0, uint32_t seed, hipStream_t s) {
    GaugeArgs a;
    a.U = static_cast<double2 *>(field);
    for (int m = 0; m < 4; ++m) a.L[m] = g.L[m];
    a.V = 2 * g.Vh;
    a.beta = beta;
    a.k0 = seed;
    a.k1 = 0x68656174u;
    a.S = size_t(g.S);
    const int nb = (g.Vh + kBlock - 1) / kBlock;
    for (int n = 0; n < nsweeps; ++n)
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par) {
                a.mu = mu;
                a.par = par;
                a.sweep = sweep0 + uint32_t(n);
                if (packed)
                    hipLaunchKernelGGL(heatbath_kernel<true>, dim3(nb), dim3(kBlock), 0, s, a);
                else
                    hipLaunchKernelGGL(heatbath_kernel<false>, dim3(nb), dim3(kBlock), 0, s, a);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

size_t plaquette_workspace_bytes(const Geom &g) {
    return sizeof(double) * size_t((2 * g.Vh + kBlock - 1) / kBlock);
}

hipError_t launch_plaquette_field(const Geom &g, const void *field, bool packed, double *out,
                                  void *work, hipStream_t s) {
    const int nb = (2 * g.Vh + kBlock - 1) / kBlock;
    if (packed)
        hipLaunchKernelGGL(plaquette_kernel<true>, dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const double2 *>(field), g, static_cast<double *>(work));
    else
        hipLaunchKernelGGL(plaquette_kernel<false>, dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const double2 *>(field), g, static_cast<double *>(work));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(plaquette_finish, dim3(1), dim3(kBlock), 0, s,
                       static_cast<const double *>(work), nb, 1.0 / (6.0 * 2 * g.Vh), out);
    return hipGetLastError();
}

hipError_t launch_heatbath(const Geom &g, void *canon, double beta, int nsweeps,
                           uint32_t sweep0, uint32_t seed, hipStream_t s) {
    return launch_heatbath_field(g, canon, false, beta, nsweeps, sweep0, seed, s);
}

hipError_t launch_plaquette(const Geom &g, const void *canon, double *out, void *work,
                            hipStream_t s) {
    return launch_plaquette_field(g, canon, false, out, work, s);
}

}  // namespace wl
