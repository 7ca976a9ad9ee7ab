/*
 * wilson_oracle.c -- plain FP64 CPU oracle for the Wilson-Dirac operator and
 * its Krylov solves.
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg call this library; the product (the HIP library and its
 * Python binding) never does. It shares no code with the HIP path.
 *
 * The paper (Sec. 3) names the objects only: the fermion matrix M of Wilson
 * fermions, its non-diagonal part ("dslash"), even-odd preconditioning, and the
 * inversion M^-1 b for point sources b(x0) (Sec. 4, Eq. 1). Everything below is
 * the textbook definition written out with no blocking, fusion or reordering:
 *
 *   D_W psi(x) = sum_mu [ f_mu(x) (1 - gamma_mu) U_mu(x)        psi(x+mu)
 *                       + b_mu(x) (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   M = 1 - kappa D_W,          M^dag = gamma5 M gamma5,
 *
 * with neighbours taken modulo the extents, f_mu(x) = phase_mu when the forward
 * hop wraps (x_mu = L_mu - 1), b_mu(x) = conj(phase_mu) when the backward hop
 * wraps (x_mu = 0), and 1 otherwise. Gamma matrices are explicit 4x4 complex
 * matrices in the Euclidean chiral basis; spin and colour are multiplied out in
 * full (no projection to half spinors).
 *
 * Layouts: complex128, site s = x + Lx*(y + Ly*(z + Lz*t));
 *   U[s][mu][a][b]  (link on the bond s -> s+mu),   psi[s][spin][colour].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* ------------------------------------------------------------------------ */
/* Dirac matrices (Euclidean, Hermitian, chiral basis):                      */
/*   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = x, y, z)              */
/*   gamma_t = [[0, 1], [1, 0]]                                              */
/*   gamma_5 = gamma_x gamma_y gamma_z gamma_t  ( = diag(1, 1, -1, -1) )     */
/* ------------------------------------------------------------------------ */
static cplx GAM[4][4][4];
static cplx GAM5[4][4];

static void matmul4(const cplx a[4][4], const cplx b[4][4], cplx c[4][4])
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
            c[i][j] = s;
        }
}

__attribute__((constructor)) static void build_gammas(void)
{
    cplx sigma[3][2][2];
    memset(sigma, 0, sizeof sigma);
    sigma[0][0][1] = 1;  sigma[0][1][0] = 1;            /* sigma_1 */
    sigma[1][0][1] = -I; sigma[1][1][0] = I;            /* sigma_2 */
    sigma[2][0][0] = 1;  sigma[2][1][1] = -1;           /* sigma_3 */

    memset(GAM, 0, sizeof GAM);
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                GAM[k][a][2 + b] = -I * sigma[k][a][b];
                GAM[k][2 + a][b] = I * sigma[k][a][b];
            }
    for (int a = 0; a < 2; ++a) {
        GAM[3][a][2 + a] = 1;
        GAM[3][2 + a][a] = 1;
    }
    cplx t1[4][4], t2[4][4];
    matmul4(GAM[0], GAM[1], t1);
    matmul4(t1, GAM[2], t2);
    matmul4(t2, GAM[3], GAM5);
}

/* Copy out the oracle's Dirac matrices: mu = 0..3 for gamma_mu, 4 for gamma_5. */
void orc_gamma(int mu, double *out /* [4][4][2] */)
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx v = (mu < 4) ? GAM[mu][i][j] : GAM5[i][j];
            out[(i * 4 + j) * 2 + 0] = creal(v);
            out[(i * 4 + j) * 2 + 1] = cimag(v);
        }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry                                                          */
/* ------------------------------------------------------------------------ */
static long volume4(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords_of(const int L[4], long s, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long index_of(const int L[4], const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* ------------------------------------------------------------------------ */
/* The hopping term D_W at one site.                                        */
/*   g5in != 0 : use (gamma5 psi) in place of psi (for M^dag = g5 M g5)      */
/*   mask_par >= 0 : treat psi as zero on sites of that parity               */
/* ------------------------------------------------------------------------ */
static void spin_apply(const cplx m[4][4], const cplx in[4][3], cplx out[4][3])
{
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) {
            cplx s = 0;
            for (int b = 0; b < 4; ++b) s += m[a][b] * in[b][i];
            out[a][i] = s;
        }
}

static void load_spinor(const cplx *psi, long s, int g5in, cplx v[4][3])
{
    cplx raw[4][3];
    memcpy(raw, psi + s * 12, sizeof raw);
    if (g5in)
        spin_apply(GAM5, raw, v);
    else
        memcpy(v, raw, sizeof raw);
}

static void hop_site(const cplx *U, const cplx *psi, const int L[4],
                     const cplx ph[4], long s, int g5in, int mask_par,
                     cplx out[4][3])
{
    int c[4];
    coords_of(L, s, c);
    memset(out, 0, sizeof(cplx) * 12);
    for (int mu = 0; mu < 4; ++mu) {
        int cf[4], cb[4];
        memcpy(cf, c, sizeof cf);
        memcpy(cb, c, sizeof cb);
        cf[mu] = (c[mu] + 1) % L[mu];
        cb[mu] = (c[mu] - 1 + L[mu]) % L[mu];
        long sf = index_of(L, cf), sb = index_of(L, cb);
        cplx pf = (c[mu] == L[mu] - 1) ? ph[mu] : 1.0;
        cplx pb = (c[mu] == 0) ? conj(ph[mu]) : 1.0;

        cplx one_minus[4][4], one_plus[4][4];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx d = (a == b) ? 1.0 : 0.0;
                one_minus[a][b] = d - GAM[mu][a][b];
                one_plus[a][b] = d + GAM[mu][a][b];
            }

        /* forward: f (1 - gamma_mu) U_mu(x) psi(x+mu) */
        {
            cplx v[4][3], w[4][3], r[4][3];
            load_spinor(psi, sf, g5in, v);
            if (mask_par >= 0 && parity_of(cf) == mask_par) memset(v, 0, sizeof v);
            const cplx *u = U + (s * 4 + mu) * 9;
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    cplx acc = 0;
                    for (int j = 0; j < 3; ++j) acc += u[i * 3 + j] * v[a][j];
                    w[a][i] = acc;
                }
            spin_apply(one_minus, w, r);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) out[a][i] += pf * r[a][i];
        }
        /* backward: b (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) */
        {
            cplx v[4][3], w[4][3], r[4][3];
            load_spinor(psi, sb, g5in, v);
            if (mask_par >= 0 && parity_of(cb) == mask_par) memset(v, 0, sizeof v);
            const cplx *u = U + (sb * 4 + mu) * 9;
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    cplx acc = 0;
                    for (int j = 0; j < 3; ++j) acc += conj(u[j * 3 + i]) * v[a][j];
                    w[a][i] = acc;
                }
            spin_apply(one_plus, w, r);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) out[a][i] += pb * r[a][i];
        }
    }
}

/* M (or M^dag = g5 M g5) at one site: out = psi(x) - kappa D_W psi(x). */
static void mop_site(const cplx *U, const cplx *psi, const int L[4],
                     const cplx ph[4], double kappa, int dagger, long s,
                     cplx out[4][3])
{
    cplx h[4][3], own[4][3], m[4][3];
    hop_site(U, psi, L, ph, s, dagger, -1, h);
    load_spinor(psi, s, dagger, own);
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) m[a][i] = own[a][i] - kappa * h[a][i];
    if (dagger)
        spin_apply(GAM5, m, out);
    else
        memcpy(out, m, sizeof m);
}

/*
 * Twisted-mass Wilson operator of one flavour (paper Sec. 3: the group's
 * N_f = 2 twisted-mass Wilson fermions; the two flavours carry +mu and -mu):
 *   M(mu) = 1 + 2 i kappa mu gamma5 - kappa D_W,
 * and its adjoint M(mu)^dag = 1 - 2 i kappa mu gamma5 - kappa D_W^dag
 * = gamma5 M(-mu) gamma5. The twist is added to the Wilson site operator.
 */
static void mop_tm_site(const cplx *U, const cplx *psi, const int L[4],
                        const cplx ph[4], double kappa, double mu, int dagger, long s,
                        cplx out[4][3])
{
    cplx w[4][3], raw[4][3], g5psi[4][3];
    mop_site(U, psi, L, ph, kappa, dagger, s, w);
    memcpy(raw, psi + s * 12, sizeof raw);
    spin_apply(GAM5, raw, g5psi);
    double tw = dagger ? -2.0 * kappa * mu : 2.0 * kappa * mu;
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) out[a][i] = w[a][i] + I * tw * g5psi[a][i];
}

/* ------------------------------------------------------------------------ */
/* Whole-lattice operators (exported)                                        */
/* ------------------------------------------------------------------------ */

/* out = D_W psi  (dagger: D_W^dag = g5 D_W g5) */
void orc_dslash(const cplx *U, const cplx *psi, cplx *out, const int L[4],
                const cplx ph[4], int dagger)
{
    long V = volume4(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        cplx h[4][3];
        hop_site(U, psi, L, ph, s, dagger, -1, h);
        if (dagger)
            spin_apply(GAM5, h, (cplx(*)[3])(out + s * 12));
        else
            memcpy(out + s * 12, h, sizeof h);
    }
}

/* out = M psi = psi - kappa D_W psi  (dagger: M^dag = g5 M g5) */
void orc_mop(const cplx *U, const cplx *psi, cplx *out, const int L[4],
             const cplx ph[4], double kappa, int dagger)
{
    long V = volume4(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s)
        mop_site(U, psi, L, ph, kappa, dagger, s, (cplx(*)[3])(out + s * 12));
}

/* out = M(mu) psi (dagger: M(mu)^dag psi), twisted-mass Wilson operator */
void orc_mop_tm(const cplx *U, const cplx *psi, cplx *out, const int L[4],
                const cplx ph[4], double kappa, double mu, int dagger)
{
    long V = volume4(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s)
        mop_tm_site(U, psi, L, ph, kappa, mu, dagger, s, (cplx(*)[3])(out + s * 12));
}

/* M (or M^dag) at a list of sites only: out[n][12]. */
void orc_mop_sites(const cplx *U, const cplx *psi, const int L[4],
                   const cplx ph[4], double kappa, int dagger,
                   const int64_t *sites, long n, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k)
        mop_site(U, psi, L, ph, kappa, dagger, (long)sites[k],
                 (cplx(*)[3])(out + k * 12));
}

/* D_W (or D_W^dag) at a list of sites only: out[n][12]. */
void orc_dslash_sites(const cplx *U, const cplx *psi, const int L[4],
                      const cplx ph[4], int dagger, const int64_t *sites,
                      long n, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        cplx h[4][3];
        hop_site(U, psi, L, ph, (long)sites[k], dagger, -1, h);
        if (dagger)
            spin_apply(GAM5, h, (cplx(*)[3])(out + k * 12));
        else
            memcpy(out + k * 12, h, sizeof h);
    }
}

/*
 * Even-odd blocks of D_W (even = (x+y+z+t) even). With out_parity p this is
 * D_{p,1-p}: the output lives on parity p and only the input on parity 1-p
 * enters; the output on parity 1-p is zero. Whole-lattice canonical arrays.
 */
void orc_dslash_eo(const cplx *U, const cplx *psi, cplx *out, const int L[4],
                   const cplx ph[4], int out_parity, int dagger)
{
    long V = volume4(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(L, s, c);
        cplx h[4][3];
        if (parity_of(c) != out_parity) {
            memset(out + s * 12, 0, sizeof h);
            continue;
        }
        hop_site(U, psi, L, ph, s, dagger, out_parity, h);
        if (dagger)
            spin_apply(GAM5, h, (cplx(*)[3])(out + s * 12));
        else
            memcpy(out + s * 12, h, sizeof h);
    }
}

/*
 * Schur complement on parity p:  Mhat = 1 - kappa^2 D_{p,1-p} D_{1-p,p}
 * (dagger: g5 Mhat g5). Whole-lattice arrays; output is zero on parity 1-p.
 * tmp and tmp2 are whole-lattice scratch arrays.
 */
static void schur_into(const cplx *U, const cplx *psi, cplx *out, const int L[4],
                       const cplx ph[4], double kappa, int parity, int dagger,
                       cplx *tmp, cplx *tmp2)
{
    long V = volume4(L);
    orc_dslash_eo(U, psi, tmp, L, ph, 1 - parity, dagger);
    orc_dslash_eo(U, tmp, tmp2, L, ph, parity, dagger);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(L, s, c);
        for (int k = 0; k < 12; ++k)
            out[s * 12 + k] = (parity_of(c) == parity)
                                  ? psi[s * 12 + k] - kappa * kappa * tmp2[s * 12 + k]
                                  : 0.0;
    }
}

void orc_schur(const cplx *U, const cplx *psi, cplx *out, const int L[4],
               const cplx ph[4], double kappa, int parity, int dagger)
{
    long V = volume4(L);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * 12 * V);
    cplx *tmp2 = (cplx *)malloc(sizeof(cplx) * 12 * V);
    schur_into(U, psi, out, L, ph, kappa, parity, dagger, tmp, tmp2);
    free(tmp);
    free(tmp2);
}

/*
 * Twisted-mass Schur complement on parity p, with A = 1 + 2 i kappa mu g5:
 *   S_p = A - kappa^2 D_{p,1-p} A^-1 D_{1-p,p}
 * (dagger: S_p^dag = A^dag - kappa^2 D^dag_{p,1-p} A^-dag D^dag_{1-p,p}, i.e.
 * mu -> -mu with the adjoint hops). A^-1 is applied as the solution of the
 * 4x4 spin system (1 + i t g5) y = v with t = 2 kappa mu, using the
 * explicit gamma5: y = (1 - i t g5) v / (1 + t^2). Whole-lattice arrays;
 * output is zero on parity 1-p.
 */
void orc_schur_tm(const cplx *U, const cplx *psi, cplx *out, const int L[4],
                  const cplx ph[4], double kappa, double mu, int parity, int dagger)
{
    long V = volume4(L);
    double t = (dagger ? -2.0 : 2.0) * kappa * mu;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * 12 * V);
    cplx *tmp2 = (cplx *)malloc(sizeof(cplx) * 12 * V);
    orc_dslash_eo(U, psi, tmp, L, ph, 1 - parity, dagger);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        cplx g5v[4][3];
        spin_apply(GAM5, (const cplx(*)[3])(tmp + s * 12), g5v);
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i)
                tmp[s * 12 + a * 3 + i] = (tmp[s * 12 + a * 3 + i] - I * t * g5v[a][i]) / (1.0 + t * t);
    }
    orc_dslash_eo(U, tmp, tmp2, L, ph, parity, dagger);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(L, s, c);
        cplx g5p[4][3];
        spin_apply(GAM5, (const cplx(*)[3])(psi + s * 12), g5p);
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) {
                long k = s * 12 + a * 3 + i;
                out[k] = (parity_of(c) == parity)
                             ? psi[k] + I * t * g5p[a][i] - kappa * kappa * tmp2[k]
                             : 0.0;
            }
    }
    free(tmp);
    free(tmp2);
}

/*
 * Meson correlators of one point-source propagator (paper Sec. 4, Eq. 1):
 *   C_Gamma(x) = - Tr( S^dag(x) g5 Gamma S(x) Gamma g5 ),
 * summed over the sites of each time slice, C_Gamma(t) = sum_xvec C(xvec, t),
 * with t counted from the source's time slice t0 (t_rel = (t - t0) mod Lt).
 * S(x) is the 12 x 12 spin-colour matrix whose column (spin b, colour c) is
 * the solution of M x = b for the point source of that spin and colour:
 * props[12][V][4][3], column index 3 b + c. The trace runs over spin and
 * colour. Gamma_n for n = 0..15 is the product g_x^n0 g_y^n1 g_z^n2 g_t^n3
 * of the oracle's Dirac matrices (bits n0..n3 of n; n = 15 is g5).
 * corr[n][t] (complex) for t = 0..Lt-1.
 */
void orc_meson(const cplx *props, const int L[4], int t0, cplx *corr)
{
    long V = volume4(L);
    int Lt = L[3];
    cplx G[16][4][4], A[16][4][4], B[16][4][4];
    for (int n = 0; n < 16; ++n) {
        cplx m[4][4], t[4][4];
        memset(m, 0, sizeof m);
        for (int i = 0; i < 4; ++i) m[i][i] = 1;
        for (int mu = 0; mu < 4; ++mu)
            if (n >> mu & 1) {
                matmul4((const cplx(*)[4])m, (const cplx(*)[4])GAM[mu], t);
                memcpy(m, t, sizeof m);
            }
        memcpy(G[n], m, sizeof m);
        matmul4((const cplx(*)[4])GAM5, (const cplx(*)[4])G[n], A[n]);   /* g5 Gamma */
        matmul4((const cplx(*)[4])G[n], (const cplx(*)[4])GAM5, B[n]);   /* Gamma g5 */
    }
    memset(corr, 0, sizeof(cplx) * 16 * Lt);
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(L, s, c);
        int tr = ((c[3] - t0) % Lt + Lt) % Lt;
        /* S[i][j]: row i = (sink spin, colour), column j = (source spin, colour) */
        cplx S[12][12];
        for (int j = 0; j < 12; ++j)
            for (int i = 0; i < 12; ++i) S[i][j] = props[((long)j * V + s) * 12 + i];
        for (int n = 0; n < 16; ++n) {
            /* SB = S (B (x) 1_colour); ASB = (A (x) 1_colour) SB;
               Tr(S^dag ASB) = sum_{i,j} conj(S[j][i]) ASB[j][i] */
            cplx SB[12][12], ASB[12][12];
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) {
                    cplx b = 0;
                    for (int k = 0; k < 4; ++k) b += S[i][k * 3 + j % 3] * B[n][k][j / 3];
                    SB[i][j] = b;
                }
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) {
                    cplx a = 0;
                    for (int k = 0; k < 4; ++k) a += A[n][i / 3][k] * SB[k * 3 + i % 3][j];
                    ASB[i][j] = a;
                }
            cplx tr_ = 0;
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) tr_ += conj(S[j][i]) * ASB[j][i];
            corr[n * Lt + tr] += -tr_;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pure-gauge update (paper Sec. 3: the heatbath that generates the gauge    */
/* configurations): Wilson plaquette action                                  */
/*   S = beta sum_P (1 - Re Tr U_P / 3),                                     */
/* Cabibbo-Marinari heatbath over the three SU(2) subgroups of each link,   */
/* each drawn with the Kennedy-Pendleton algorithm.                          */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter c[4], key k[2].
   Ten rounds of two 32x32 -> 64 multiplications with the Weyl-sequence key
   schedule between rounds. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* four uniforms in (0, 1): (x + 1/2) / 2^32 of the four Philox words */
static void uniforms4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                      const uint32_t key[2], double u[4])
{
    uint32_t ctr[4] = {a, b, c, d}, o[4];
    orc_philox(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = ((double)o[i] + 0.5) / 4294967296.0;
}

/* x0 in [-1, 1] with density ~ sqrt(1 - x0^2) exp(alpha x0), alpha >= 0, by
   rejection. For alpha >= 1 the Kennedy-Pendleton candidate:
   lambda^2 = -(ln r1 + cos^2(2 pi r2) ln r3) / (2 alpha), accepted when
   r4^2 <= 1 - lambda^2, x0 = 1 - 2 lambda^2. For alpha < 1, where that
   candidate is seldom accepted (3.6 % of attempts at alpha = 0.1), the first
   coordinate of a uniform point of the unit disk, x0 = sqrt(r1) cos(2 pi r2)
   (density ~ sqrt(1 - x0^2)), accepted when r3 <= exp(alpha (x0 - 1)).
   Either way an attempt is accepted with probability >= 0.41, so all
   HB_MAX_TRIES attempts fail with probability below 1e-29. Attempt n draws
   its four uniforms from the counter (site, tag + 16 n, sweep, 0). Returns 0
   and sets *x0 when accepted, else -1. */
#define HB_MAX_TRIES 128
static int kp_draw(double alpha, uint32_t site, uint32_t tag, uint32_t sweep,
                   const uint32_t key[2], double *x0)
{
    for (uint32_t n = 0; n < HB_MAX_TRIES; ++n) {
        double u[4];
        uniforms4(site, tag + 16u * n, sweep, 0u, key, u);
        if (alpha < 1.0) {
            double x = sqrt(u[0]) * cos(2.0 * M_PI * u[1]);
            if (u[2] <= exp(alpha * (x - 1.0))) {
                *x0 = x;
                return 0;
            }
            continue;
        }
        double c = cos(2.0 * M_PI * u[1]);
        double l2 = -(log(u[0]) + c * c * log(u[2])) / (2.0 * alpha);
        if (u[3] * u[3] <= 1.0 - l2) {
            *x0 = 1.0 - 2.0 * l2;
            return 0;
        }
    }
    return -1;
}

/* Samples of the x0 draw for one alpha (to pin its density); 2 marks a draw
   that found no accepted candidate. */
void orc_kp_samples(double alpha, int n, uint32_t seed, double *out)
{
    uint32_t key[2] = {seed, 0x6b707070u};
    for (int i = 0; i < n; ++i) {
        double x0 = 2.0;
        if (kp_draw(alpha, (uint32_t)i, 0u, 0u, key, &x0) != 0) x0 = 2.0;
        out[i] = x0;
    }
}

static void su3_mul(const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + j];
            c[i * 3 + j] = s;
        }
}

static void su3_mul_dag(const cplx *a, const cplx *b, cplx *c) /* a b^dag */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * conj(b[j * 3 + k]);
            c[i * 3 + j] = s;
        }
}

static void su3_dag_mul(const cplx *a, const cplx *b, cplx *c) /* a^dag b */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += conj(a[k * 3 + i]) * b[k * 3 + j];
            c[i * 3 + j] = s;
        }
}

static long shift(const int L[4], const int c[4], int mu, int d)
{
    int e[4] = {c[0], c[1], c[2], c[3]};
    e[mu] = (e[mu] + d + L[mu]) % L[mu];
    return index_of(L, e);
}

/* Sum of the six staples of U_mu(x), so that the action's part with this
   link is -(beta / 3) Re Tr(U_mu(x) A):
     A = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                      + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)      */
static void staple_sum(const cplx *U, const int L[4], long s, int mu, cplx A[9])
{
    int c[4];
    coords_of(L, s, c);
    memset(A, 0, sizeof(cplx) * 9);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        long xpmu = shift(L, c, mu, 1), xpnu = shift(L, c, nu, 1), xmnu = shift(L, c, nu, -1);
        int cm[4];
        coords_of(L, xmnu, cm);
        long xpmu_mnu = shift(L, cm, mu, 1);
        cplx t1[9], t2[9], m[9];
        /* upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
        su3_mul_dag(U + (xpmu * 4 + nu) * 9, U + (xpnu * 4 + mu) * 9, t1);
        su3_mul_dag(t1, U + (s * 4 + nu) * 9, t2);
        for (int k = 0; k < 9; ++k) A[k] += t2[k];
        /* lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
                = (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu) */
        su3_mul(U + (xmnu * 4 + mu) * 9, U + (xpmu_mnu * 4 + nu) * 9, m);
        su3_dag_mul(m, U + (xmnu * 4 + nu) * 9, t2);
        for (int k = 0; k < 9; ++k) A[k] += t2[k];
    }
}

/* One heatbath update of U_mu(x) (Cabibbo-Marinari): for the SU(2)
   subgroups on rows/columns (0,1), (1,2), (0,2) in turn, with W = U A and w
   its 2 x 2 block, Re Tr(r w) = 2 (r . b) for an SU(2) element
   r = [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]] and
     b = (Re(w00 + w11), -Im(w01 + w10), Re(w10 - w01), -Im(w00 - w11)) / 2.
   With k = |b| and V the SU(2) element of b / k, r = X V where X has the
   density exp(alpha X0) on SU(2), alpha = 2 beta k / 3: X0 from the
   Kennedy-Pendleton draw, (X1, X2, X3) uniform on the sphere of radius
   sqrt(1 - X0^2) (cos theta = 2 u - 1, phi = 2 pi v from the counter
   (site, tag, sweep, 1)). Then U <- R U, R = r on rows (i, j). A subgroup
   whose draw is not accepted within HB_MAX_TRIES attempts is left as it is.
   A staple term with k = 0 leaves V undefined and the density of r flat:
   r = X with alpha = 0 (Haar-uniform). */
static void hb_link(cplx *U, const int L[4], long s, int mu, double beta,
                    uint32_t sweep, const uint32_t key[2])
{
    static const int SUB[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    cplx A[9];
    staple_sum(U, L, s, mu, A);
    cplx *u = U + (s * 4 + mu) * 9;
    for (int g = 0; g < 3; ++g) {
        int i = SUB[g][0], j = SUB[g][1];
        cplx W[9];
        su3_mul(u, A, W);
        cplx w00 = W[i * 3 + i], w01 = W[i * 3 + j], w10 = W[j * 3 + i], w11 = W[j * 3 + j];
        double b0 = creal(w00 + w11) / 2, b1 = -cimag(w01 + w10) / 2;
        double b2 = creal(w10 - w01) / 2, b3 = -cimag(w00 - w11) / 2;
        double k = sqrt(b0 * b0 + b1 * b1 + b2 * b2 + b3 * b3);
        if (!(k > 0.0)) {   /* V = 1 */
            k = 0.0;
            b0 = 1.0; b1 = b2 = b3 = 0.0;
        }
        uint32_t tag = (uint32_t)mu | ((uint32_t)g << 2);
        double x0;
        if (kp_draw(2.0 * beta * k / 3.0, (uint32_t)s, tag, sweep, key, &x0) != 0) continue;
        double d[4];
        uniforms4((uint32_t)s, tag, sweep, 1u, key, d);
        double ct = 2.0 * d[0] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double ph = 2.0 * M_PI * d[1], rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
        double x1 = rad * st * cos(ph), x2 = rad * st * sin(ph), x3 = rad * ct;
        double n = k > 0.0 ? k : 1.0;
        double v0 = b0 / n, v1 = b1 / n, v2 = b2 / n, v3 = b3 / n;
        cplx X[4] = {x0 + I * x3, x2 + I * x1, -x2 + I * x1, x0 - I * x3};
        cplx Vm[4] = {v0 + I * v3, v2 + I * v1, -v2 + I * v1, v0 - I * v3};
        cplx r[4] = {X[0] * Vm[0] + X[1] * Vm[2], X[0] * Vm[1] + X[1] * Vm[3],
                     X[2] * Vm[0] + X[3] * Vm[2], X[2] * Vm[1] + X[3] * Vm[3]};
        for (int col = 0; col < 3; ++col) {
            cplx ui = u[i * 3 + col], uj = u[j * 3 + col];
            u[i * 3 + col] = r[0] * ui + r[1] * uj;
            u[j * 3 + col] = r[2] * ui + r[3] * uj;
        }
    }
}

/* nsweeps heatbath sweeps at coupling beta, sweep numbers sweep0, sweep0+1, ...
   (part of every random counter); within a sweep the links of direction mu
   on the even, then the odd sites, for mu = 0..3 (links of one direction and
   parity do not enter each other's staples, so their order is free). */
void orc_heatbath(cplx *U, const int L[4], double beta, int nsweeps, uint32_t sweep0,
                  uint32_t seed)
{
    long V = volume4(L);
    uint32_t key[2] = {seed, 0x68656174u};
    for (int n = 0; n < nsweeps; ++n)
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par) {
#pragma omp parallel for schedule(static)
                for (long s = 0; s < V; ++s) {
                    int c[4];
                    coords_of(L, s, c);
                    if (parity_of(c) == par) hb_link(U, L, s, mu, beta, sweep0 + (uint32_t)n, key);
                }
            }
}

/* Mean plaquette: average over sites and the 6 planes of Re tr(U_mu nu)/3. */
double orc_plaquette(const cplx *U, const int L[4])
{
    long V = volume4(L);
    double sum = 0;
#pragma omp parallel for schedule(static) reduction(+ : sum)
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(L, s, c);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                int cm[4], cn[4];
                memcpy(cm, c, sizeof cm);
                memcpy(cn, c, sizeof cn);
                cm[mu] = (c[mu] + 1) % L[mu];
                cn[nu] = (c[nu] + 1) % L[nu];
                const cplx *a = U + (s * 4 + mu) * 9;                 /* U_mu(x)      */
                const cplx *b = U + (index_of(L, cm) * 4 + nu) * 9;   /* U_nu(x+mu)   */
                const cplx *e = U + (index_of(L, cn) * 4 + mu) * 9;   /* U_mu(x+nu)   */
                const cplx *d = U + (s * 4 + nu) * 9;                 /* U_nu(x)      */
                cplx ab[9], abe[9], tr = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        cplx acc = 0;
                        for (int k = 0; k < 3; ++k) acc += a[i * 3 + k] * b[k * 3 + j];
                        ab[i * 3 + j] = acc;
                    }
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        cplx acc = 0;
                        for (int k = 0; k < 3; ++k) acc += ab[i * 3 + k] * conj(e[j * 3 + k]);
                        abe[i * 3 + j] = acc;
                    }
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) tr += abe[i * 3 + k] * conj(d[i * 3 + k]);
                sum += creal(tr) / 3.0;
            }
    }
    return sum / (6.0 * V);
}

/* ------------------------------------------------------------------------ */
/* Vector helpers (whole-lattice, n complex entries)                         */
/* ------------------------------------------------------------------------ */
static double vnorm2(const cplx *a, long n)
{
    double s = 0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

static cplx vdot(const cplx *a, const cplx *b, long n) /* sum conj(a) b */
{
    double re = 0, im = 0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (long i = 0; i < n; ++i) {
        cplx v = conj(a[i]) * b[i];
        re += creal(v);
        im += cimag(v);
    }
    return re + I * im;
}

/* ------------------------------------------------------------------------ */
/* Solvers                                                                   */
/* ------------------------------------------------------------------------ */
/* A solve gives up after this many true-residual restarts (status 1). */
#define ORC_MAX_RESTARTS 64

typedef struct {
    int32_t iterations;  /* Krylov iterations over all restarts */
    int32_t restarts;    /* true-residual restarts */
    double true_res;     /* ||b - M x|| / ||b|| recomputed at the end */
} orc_stats;

/*
 * CG on the normal equations M^dag M x = M^dag b (Hestenes-Stiefel), x0 = x
 * on entry. The CG loop stops when ||r_k|| <= eta ||M^dag b||; then the true
 * residual rho = ||b - M x|| / ||b|| is recomputed, and CG restarts from x with
 * eta <- eta * (tol / rho) / 2 until rho <= tol.
 * Returns 0 when rho <= tol, 1 when maxiter (or the restart limit) was reached
 * first, 2 when the residual is not finite.
 */
int orc_cgnr(const cplx *U, const cplx *b, cplx *x, const int L[4],
             const cplx ph[4], double kappa, double tol, int maxiter,
             orc_stats *st)
{
    long n = volume4(L) * 12;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *t = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    double bnorm = sqrt(vnorm2(b, n));
    orc_mop(U, b, t, L, ph, kappa, 1);
    double mbnorm = sqrt(vnorm2(t, n));
    double eta = tol;
    int it = 0, restarts = 0, status = 1;
    double rho = 1.0;
    for (;;) {
        orc_mop(U, x, t, L, ph, kappa, 0);
        for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];
        orc_mop(U, t, r, L, ph, kappa, 1);
        memcpy(p, r, sizeof(cplx) * n);
        double rr = vnorm2(r, n);
        while (rr > eta * eta * mbnorm * mbnorm && it < maxiter) {
            orc_mop(U, p, t, L, ph, kappa, 0);
            double pap = vnorm2(t, n);
            if (!(pap > 0.0) || !isfinite(pap)) break;
            double alpha = rr / pap;
            orc_mop(U, t, q, L, ph, kappa, 1);
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            double rr_new = vnorm2(r, n);
            double beta = rr_new / rr;
            rr = rr_new;
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            ++it;
        }
        orc_mop(U, x, t, L, ph, kappa, 0);
        for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];
        rho = sqrt(vnorm2(t, n)) / bnorm;
        if (!isfinite(rho)) { status = 2; break; }
        if (rho <= tol) { status = 0; break; }
        if (it >= maxiter || restarts >= ORC_MAX_RESTARTS) { status = 1; break; }
        eta = eta * (tol / rho) * 0.5;
        ++restarts;
    }
    if (st) { st->iterations = it; st->restarts = restarts; st->true_res = rho; }
    free(r); free(p); free(t); free(q);
    return status;
}

/*
 * CGNR for the twisted-mass operator: orc_cgnr's algorithm (CG on
 * M^dag M x = M^dag b, true-residual restarts) with M = M(mu).
 */
int orc_cgnr_tm(const cplx *U, const cplx *b, cplx *x, const int L[4],
                const cplx ph[4], double kappa, double mu, double tol, int maxiter,
                orc_stats *st)
{
    long n = volume4(L) * 12;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *t = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    double bnorm = sqrt(vnorm2(b, n));
    orc_mop_tm(U, b, t, L, ph, kappa, mu, 1);
    double mbnorm = sqrt(vnorm2(t, n));
    double eta = tol;
    int it = 0, restarts = 0, status = 1;
    double rho = 1.0;
    for (;;) {
        orc_mop_tm(U, x, t, L, ph, kappa, mu, 0);
        for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];
        orc_mop_tm(U, t, r, L, ph, kappa, mu, 1);
        memcpy(p, r, sizeof(cplx) * n);
        double rr = vnorm2(r, n);
        while (rr > eta * eta * mbnorm * mbnorm && it < maxiter) {
            orc_mop_tm(U, p, t, L, ph, kappa, mu, 0);
            double pap = vnorm2(t, n);
            if (!(pap > 0.0) || !isfinite(pap)) break;
            double alpha = rr / pap;
            orc_mop_tm(U, t, q, L, ph, kappa, mu, 1);
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            double rr_new = vnorm2(r, n);
            double beta = rr_new / rr;
            rr = rr_new;
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            ++it;
        }
        orc_mop_tm(U, x, t, L, ph, kappa, mu, 0);
        for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];
        rho = sqrt(vnorm2(t, n)) / bnorm;
        if (!isfinite(rho)) { status = 2; break; }
        if (rho <= tol) { status = 0; break; }
        if (it >= maxiter || restarts >= ORC_MAX_RESTARTS) { status = 1; break; }
        eta = eta * (tol / rho) * 0.5;
        ++restarts;
    }
    if (st) { st->iterations = it; st->restarts = restarts; st->true_res = rho; }
    free(r); free(p); free(t); free(q);
    return status;
}

/*
 * Even-odd CGNR: the same Hestenes-Stiefel CG, run on the Schur system of the
 * even sites (paper Sec. 3, even-odd preconditioning). With
 *   Mhat = 1 - kappa^2 D_eo D_oe   and   bhat_e = b_e + kappa D_eo b_o,
 * CG solves Mhat^dag Mhat x_e = Mhat^dag bhat_e from x_e (the even part of x
 * on entry); the odd part then follows exactly from the odd rows of M x = b:
 *   x_o = b_o + kappa D_oe x_e.
 * Stopping and restarts as in orc_cgnr: the CG loop stops when
 * ||r_k|| <= eta ||Mhat^dag bhat_e||, the true residual ||b - M x|| / ||b|| of
 * the full system is recomputed, and CG restarts from x_e with
 * eta <- eta (tol / rho) / 2 until rho <= tol. Same return codes as orc_cgnr.
 * All arrays are whole-lattice; the Krylov vectors are zero on odd sites.
 */
int orc_cgnr_eo(const cplx *U, const cplx *b, cplx *x, const int L[4],
                const cplx ph[4], double kappa, double tol, int maxiter,
                orc_stats *st)
{
    long V = volume4(L), n = V * 12;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *t = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    cplx *bh = malloc(sizeof(cplx) * n), *xe = malloc(sizeof(cplx) * n);
    cplx *w1 = malloc(sizeof(cplx) * n), *w2 = malloc(sizeof(cplx) * n);
    char *even = malloc(V);
    for (long s = 0; s < V; ++s) {
        int c[4];
        coords_of(L, s, c);
        even[s] = parity_of(c) == 0;
    }
    double bnorm = sqrt(vnorm2(b, n));
    /* bhat_e = b_e + kappa D_eo b  (only the odd part of b enters D_eo) */
    orc_dslash_eo(U, b, w1, L, ph, 0, 0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) bh[i] = even[i / 12] ? b[i] + kappa * w1[i] : 0.0;
    schur_into(U, bh, t, L, ph, kappa, 0, 1, w1, w2);
    double mbnorm = sqrt(vnorm2(t, n));
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) xe[i] = even[i / 12] ? x[i] : 0.0;
    double eta = tol;
    int it = 0, restarts = 0, status = 1;
    double rho = 1.0;
    for (;;) {
        /* r = Mhat^dag (bhat - Mhat x_e); p = r */
        schur_into(U, xe, t, L, ph, kappa, 0, 0, w1, w2);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) t[i] = bh[i] - t[i];
        schur_into(U, t, r, L, ph, kappa, 0, 1, w1, w2);
        memcpy(p, r, sizeof(cplx) * n);
        double rr = vnorm2(r, n);
        while (rr > eta * eta * mbnorm * mbnorm && it < maxiter) {
            schur_into(U, p, t, L, ph, kappa, 0, 0, w1, w2);
            double pap = vnorm2(t, n);
            if (!(pap > 0.0) || !isfinite(pap)) break;
            double alpha = rr / pap;
            schur_into(U, t, q, L, ph, kappa, 0, 1, w1, w2);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) {
                xe[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            double rr_new = vnorm2(r, n);
            double beta = rr_new / rr;
            rr = rr_new;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            ++it;
        }
        /* x = (x_e, b_o + kappa D_oe x_e) */
        orc_dslash_eo(U, xe, w1, L, ph, 1, 0);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) x[i] = even[i / 12] ? xe[i] : b[i] + kappa * w1[i];
        orc_mop(U, x, t, L, ph, kappa, 0);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];
        rho = sqrt(vnorm2(t, n)) / bnorm;
        if (!isfinite(rho)) { status = 2; break; }
        if (rho <= tol) { status = 0; break; }
        if (it >= maxiter || restarts >= ORC_MAX_RESTARTS) { status = 1; break; }
        eta = eta * (tol / rho) * 0.5;
        ++restarts;
    }
    if (st) { st->iterations = it; st->restarts = restarts; st->true_res = rho; }
    free(r); free(p); free(t); free(q); free(bh); free(xe); free(w1); free(w2); free(even);
    return status;
}

/*
 * Plain Lanczos tridiagonalisation of A = M^dag M from the unit start vector
 * v (overwritten), no reorthogonalisation: for k = 0, 1, ...
 *   w = A v_k - beta_{k-1} v_{k-1},  alpha_k = <v_k, w>,  w -= alpha_k v_k,
 *   beta_k = ||w||,  v_{k+1} = w / beta_k.
 * alpha[0..n) and beta[0..n-1) receive the tridiagonal matrix T (n returned,
 * n <= steps; it stops early when beta_k <= 1e-13 |alpha_k|, an invariant
 * subspace, where T is exact). The extreme eigenvalues of T approximate
 * sigma_max^2 and sigma_min^2 of M from inside the spectrum.
 */
int orc_lanczos_mdm(const cplx *U, cplx *v, const int L[4], const cplx ph[4],
                    double kappa, int steps, double *alpha, double *beta)
{
    long n = volume4(L) * 12;
    cplx *vp = calloc(n, sizeof(cplx)), *t = malloc(sizeof(cplx) * n);
    cplx *w = malloc(sizeof(cplx) * n);
    double bprev = 0.0;
    int k = 0;
    for (; k < steps; ++k) {
        orc_mop(U, v, t, L, ph, kappa, 0);
        orc_mop(U, t, w, L, ph, kappa, 1);
        double a = creal(vdot(v, w, n));
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) w[i] = w[i] - a * v[i] - bprev * vp[i];
        alpha[k] = a;
        double bk = sqrt(vnorm2(w, n));
        if (bk <= 1e-13 * fabs(a)) { ++k; break; }
        if (k + 1 < steps) beta[k] = bk;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            vp[i] = v[i];
            v[i] = w[i] / bk;
        }
        bprev = bk;
    }
    free(vp); free(t); free(w);
    return k;
}

/*
 * BiCGStab on M x = b (van der Vorst 1992), x0 = x on entry, shadow residual
 * rhat = r0. Stops on ||r|| / ||b|| <= tol, then recomputes the true residual;
 * when that misses tol, or rho or omega vanish, it restarts from x with
 * rhat = r. Returns 0 when the true residual is <= tol, 1 at maxiter (or the
 * restart limit), 2 when the residual is not finite.
 */
int orc_bicgstab(const cplx *U, const cplx *b, cplx *x, const int L[4],
                 const cplx ph[4], double kappa, double tol, int maxiter,
                 orc_stats *st)
{
    long n = volume4(L) * 12;
    cplx *r = malloc(sizeof(cplx) * n), *rh = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n), *v = malloc(sizeof(cplx) * n);
    cplx *s = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    double bnorm = sqrt(vnorm2(b, n));
    int it = 0, passes = 0, status = 1;
    double res = 1.0;
    for (;;) {
        orc_mop(U, x, t, L, ph, kappa, 0);
        for (long i = 0; i < n; ++i) r[i] = b[i] - t[i];
        res = sqrt(vnorm2(r, n)) / bnorm;
        if (!isfinite(res)) { status = 2; break; }
        if (res <= tol) { status = 0; break; }
        if (it >= maxiter || passes > ORC_MAX_RESTARTS) { status = 1; break; }
        ++passes;
        memcpy(rh, r, sizeof(cplx) * n);
        memset(p, 0, sizeof(cplx) * n);
        memset(v, 0, sizeof(cplx) * n);
        cplx rho_old = 1, alpha = 1, omega = 1;
        while (it < maxiter) {
            cplx rho = vdot(rh, r, n);
            if (cabs(rho) == 0.0 || cabs(omega) == 0.0) break;
            cplx beta = (rho / rho_old) * (alpha / omega);
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            orc_mop(U, p, v, L, ph, kappa, 0);
            cplx rv = vdot(rh, v, n);
            if (cabs(rv) == 0.0) break;
            alpha = rho / rv;
            for (long i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            ++it;
            if (sqrt(vnorm2(s, n)) <= tol * bnorm) {
                for (long i = 0; i < n; ++i) x[i] += alpha * p[i];
                break;
            }
            orc_mop(U, s, t, L, ph, kappa, 0);
            double tt = vnorm2(t, n);
            if (tt == 0.0) break;
            omega = vdot(t, s, n) / tt;
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * p[i] + omega * s[i];
                r[i] = s[i] - omega * t[i];
            }
            rho_old = rho;
            if (sqrt(vnorm2(r, n)) <= tol * bnorm) break;
        }
    }
    if (st) { st->iterations = it; st->restarts = passes > 0 ? passes - 1 : 0; st->true_res = res; }
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return status;
}
