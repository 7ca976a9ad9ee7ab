/*
 * wilson.h -- C ABI of libwilson.so: the Wilson-Dirac fermion matrix and its
 * Krylov solves on one AMD Instinct MI355X (gfx950).
 *
 * The problem (paper, Sec. 3 and Sec. 4): the fermion matrix of Wilson-type
 * fermions, M = 1 - kappa D_W, whose non-diagonal part D_W ("dslash") is the
 * 8-neighbour SU(3) x spin hopping stencil
 *
 *   D_W psi(x) = sum_mu [ f_mu(x) (1 - gamma_mu) U_mu(x)        psi(x+mu)
 *                       + b_mu(x) (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ],
 *
 * even-odd preconditioning of M, and the inversion x = M^-1 b (the point-source
 * propagators of Eq. 1 are 12 such solves). The paper does not print these
 * formulas; this library uses the standard definitions:
 *   - Euclidean chiral gamma basis, gamma_5 = gamma_x gamma_y gamma_z gamma_t
 *     = diag(1, 1, -1, -1); M^dag = gamma_5 M gamma_5;
 *   - boundary phases: a forward hop that wraps (x_mu = L_mu - 1) is multiplied
 *     by phase_mu, a backward hop that wraps (x_mu = 0) by conj(phase_mu); the
 *     usual choice is (1, 1, 1, -1): periodic in space, antiperiodic in time.
 *   - even sites: (x + y + z + t) even. Schur complement on parity p:
 *     Mhat_p = 1 - kappa^2 D_{p,1-p} D_{1-p,p}.
 *
 * Lattice: dims = {Lx, Ly, Lz, Lt}; every extent must be even and >= 2 (the
 * even-odd layout needs it). Canonical site index s = x + Lx*(y + Ly*(z + Lz*t)).
 *
 * Buffers and ownership. Every data pointer is DEVICE memory owned by the
 * caller; the library borrows it for stream-ordered work and keeps no
 * reference after the call's work completes. Kernels run on the HIP stream
 * passed as `stream` (a hipStream_t; NULL = the null stream); the dslash calls
 * return as soon as the work is enqueued, the solvers return after it is done.
 * Nothing may alias: in != out, b != x, and no buffer may overlap `work`.
 *
 * Packed layouts ("WL layout"), produced by wl_pack_* and consumed by every
 * operator and solver. With Vh = V/2 and S = Vh rounded up to a multiple of 64:
 *   spinor (full field): [parity][chunk][S], parity 0 = even block first;
 *     a half field (one parity) is one [chunk][S] block, wl_spinor_bytes(.., 1).
 *     FP64: 12 chunks of double2 (one complex each, index spin*3 + colour);
 *     FP32: 6 chunks of float4 (two consecutive complex components each);
 *     FP16 (WL_F16S): 3 chunks of 8 binary16 values holding psi/s, where
 *     s = 2^e is the power of two with m = f 2^e, f in [0.5, 1), m = max |real
 *     or imaginary component| of the site (s = 1 for a zero site), followed by
 *     the S FP32 scales s of the block (52 bytes per site).
 *   gauge: [parity][mu][chunk][S]; link U_mu(x) stored at the parity and
 *     checkerboard index of x. 18-real: the 9 complex entries, row-major;
 *     12-real (WL_LINK12): rows 0 and 1 only, row 2 = conj(row0 x row1) is
 *     rebuilt in the kernel (exact for det U = 1). FP64: one complex per
 *     double2 chunk; FP32: float4 chunks of two complex, and for 18-real a
 *     last float2 chunk with the ninth; FP16 (unscaled, |U_ij| <= 1): chunks
 *     of four complex (8 binary16), then the rest in one narrower chunk
 *     (18-real: 2 chunks + one complex; 12-real: 1 chunk + two complex).
 *   Checkerboard index of site s (with parity (x+y+z+t) & 1) is s / 2.
 *   Padding entries (checkerboard index >= Vh) are never read or written by
 *   the operators.
 *
 * Errors: 0 = WL_OK; positive = a solve finished without reaching tol (x holds
 * the best iterate seen, stats->true_res is set); negative = nothing was done.
 * No exceptions cross the ABI. wl_last_error() returns a thread-local message
 * for the last non-zero return on the calling thread.
 */
#ifndef WILSON_H
#define WILSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- flags --------------------------------------------------------------- */
#define WL_F64        0x0u   /* storage and arithmetic precision: FP64        */
#define WL_F32        0x1u   /* FP32                                          */
#define WL_F16S       0x2u   /* FP16 storage (spinors scaled per site), FP32
                                arithmetic                                    */
#define WL_PREC_MASK  0x3u
#define WL_LINK18     0x0u   /* links stored as 18 reals                      */
#define WL_LINK12     0x4u   /* links stored as 12 reals (rows 0, 1)          */
#define WL_DAG        0x8u   /* apply the adjoint (M^dag, D_W^dag, Mhat^dag)  */
#define WL_HOP        0x10u  /* return the hopping term only (no 1 - kappa.)  */
#define WL_EO         0x20u  /* solvers: even-odd (Schur) preconditioning     */
#define WL_MIXED      0x40u  /* solvers: low-precision inner Krylov iterations
                                (WL_F32, the default, or WL_F16S) inside an
                                FP64 outer loop                               */
#define WL_X0         0x80u  /* solvers: x holds the initial guess            */
#define WL_GRAPH      0x100u /* solvers: capture each chunk of Krylov
                                iterations once into a HIP graph and replay
                                it (fewer launch overheads on small
                                lattices); the solve waits for `stream` to
                                drain, then runs on a library-owned stream */
#define WL_CANON      0x200u /* solve_cg, solve_bicgstab and their twisted-
                                mass forms: gauge, b and x are in the
                                canonical complex128 layouts (those
                                wl_pack_gauge / wl_pack_spinor read); the
                                solve packs them into its workspace and
                                unpacks x at the end                          */

/* ---- environment ----------------------------------------------------------
 * WL_TUNE=0             no autotuning of launch shapes (see wl_tuning_report)
 * WL_TUNE_FILE=path     keep the autotuner's choices in this file
 * WL_TUNE_FORCE=n,c,g   impose one launch shape on every hop launch (testing)
 * WL_DELTA_F32=d        reliable-update threshold of FP32-inner mixed CG
 *                       (default 1e-4); WL_DELTA_F16 likewise (default 0.2);
 *                       WL_DELTA_BI_F32 / WL_DELTA_BI_F16 for mixed BiCGStab
 *                       (defaults 0.1 / 0.3)
 * WL_TRACE=1            one line per solver pass on stderr
 * None of these changes a result's bits except the WL_DELTA_* thresholds.  */

/* ---- status codes -------------------------------------------------------- */
#define WL_OK          0
#define WL_NOCONV      1     /* maxiter reached                               */
#define WL_BREAKDOWN   2     /* a Krylov scalar vanished or became non-finite */
#define WL_STAGNATED   3     /* no new best residual for a long stretch       */
#define WL_EINVAL     (-1)   /* bad dims, phases, flags, null or aliasing     */
#define WL_EWORKSPACE (-2)   /* work_bytes < wl_workspace_bytes(...)          */
#define WL_EHIP       (-3)   /* a HIP runtime call failed                     */

typedef struct {
    int32_t status;           /* same value the solver returned               */
    int32_t iterations;       /* Krylov iterations over all restarts          */
    int32_t restarts;         /* true-residual restarts / outer corrections   */
    int32_t reliable_updates; /* FP64 refreshes inside mixed-precision CG     */
    double true_res;          /* ||b - M x|| / ||b||, FP64, full lattice      */
    double seconds;           /* wall time of the solve                       */
    double flops;             /* model flops (1320/site per D_W)              */
    double bytes;             /* algorithmic bytes moved by all kernels       */
    int32_t fp64_iterations;  /* Krylov iterations run in FP64: all of them
                                 without WL_MIXED; with it, those of a mixed
                                 BiCGStab that continued in FP64 after its
                                 low-precision sequence stalled (0 for CG)    */
    int32_t reserved;         /* 0                                            */
} wl_solve_stats;

/* Library version string and the thread-local message of the last error. */
const char *wl_version(void);
const char *wl_last_error(void);

/* Bytes of a packed spinor with `nparity` (1 = half field, 2 = full field)
 * parity blocks, or of a packed gauge field, for the precision and link format
 * in `flags`. Returns 0 for invalid dims. */
size_t wl_spinor_bytes(const int32_t dims[4], uint32_t flags, int32_t nparity);
size_t wl_gauge_bytes(const int32_t dims[4], uint32_t flags);

/* Canonical -> packed gauge field. `canon` is complex128 U[V][4][3][3] on the
 * device (U[s][mu] on the bond s -> s+mu); `packed` receives
 * wl_gauge_bytes(dims, flags) bytes in the precision and link format of
 * `flags`. Asynchronous on `stream`. */
int wl_pack_gauge(const void *canon, void *packed, const int32_t dims[4],
                  uint32_t flags, void *stream);
/* Packed -> canonical: the inverse of wl_pack_gauge (FP64 18-real exactly; a
 * 12-real field gets its third rows rebuilt as conj(row0 x row1); FP32 and
 * FP16 values widened to FP64), e.g. to store a configuration the packed heat
 * bath produced. Asynchronous on `stream`. */
int wl_unpack_gauge(const void *packed, void *canon, const int32_t dims[4],
                    uint32_t flags, void *stream);

/* Canonical complex128 psi[V][4][3] <-> packed full spinor in the precision of
 * `flags`. Asynchronous on `stream`. */
int wl_pack_spinor(const void *canon, void *packed, const int32_t dims[4],
                   uint32_t flags, void *stream);
int wl_unpack_spinor(const void *packed, void *canon, const int32_t dims[4],
                     uint32_t flags, void *stream);

/* Full-lattice operator (paper Sec. 3, "dslash"; the fermion matrix M).
 *   default:          out = M psi       = psi - kappa D_W psi
 *   WL_HOP:           out = D_W psi
 *   WL_DAG:           adjoint of the above (gamma_5-conjugate)
 * `gauge` packed per flags; `in`, `out` packed full spinors in the same
 * precision. phases = {re0, im0, re1, im1, re2, im2, re3, im3}, |phase| = 1.
 * Asynchronous on `stream`; returns WL_EINVAL without enqueuing anything on a
 * bad argument. */
int wilson_dslash(const void *gauge, const void *in, void *out,
                  const int32_t dims[4], double kappa, const double phases[8],
                  uint32_t flags, void *stream);

/* Even-odd operator (paper Sec. 3: the even-odd preconditioned dslash).
 *   WL_HOP:   out (half field, parity out_parity)
 *               = D_{p,1-p} in   (in: half field of parity 1 - out_parity)
 *   default:  the Schur complement Mhat_p = 1 - kappa^2 D_{p,1-p} D_{1-p,p}
 *             on p = out_parity. `in` is a half field of parity p and `out`
 *             a FULL field (wl_spinor_bytes(dims, flags, 2) bytes): its
 *             parity-p block receives Mhat_p in, and its parity-(1-p) block
 *             is overwritten with the intermediate D_{1-p,p} in. The library
 *             allocates nothing; `in` must not overlap either block of out.
 *   WL_DAG:   adjoint of the above.
 * Asynchronous on `stream`. */
int wilson_dslash_eo(const void *gauge, const void *in, void *out,
                     const int32_t dims[4], double kappa,
                     const double phases[8], int32_t out_parity,
                     uint32_t flags, void *stream);

/* Twisted-mass Wilson fermions (paper Sec. 3: the group's N_f = 2 twisted-mass
 * Wilson action; one flavour, the other is mu -> -mu):
 *   M(mu) = 1 + 2 i kappa mu gamma_5 - kappa D_W,
 *   M(mu)^dag = 1 - 2 i kappa mu gamma_5 - kappa D_W^dag = gamma_5 M(-mu) gamma_5.
 * wilson_dslash_tm: the modes of wilson_dslash for M(mu) (WL_HOP returns D_W,
 * independent of mu). wilson_dslash_eo_tm: WL_HOP as wilson_dslash_eo; the
 * default mode is the Schur complement on p = out_parity of the diagonal
 * A = 1 + 2 i kappa mu gamma_5,
 *   S_p = A - kappa^2 D_{p,1-p} A^-1 D_{1-p,p},
 *   A^-1 = (1 - 2 i kappa mu gamma_5) / (1 + 4 kappa^2 mu^2),
 * with `out` a full field as for wilson_dslash_eo (its parity-(1-p) block
 * receives A^-1 D_{1-p,p} in); WL_DAG gives S_p^dag. mu = 0 gives exactly the
 * Wilson calls. Arguments, layouts and errors otherwise as for the Wilson
 * entry points; WL_EINVAL when mu is not finite. */
int wilson_dslash_tm(const void *gauge, const void *in, void *out,
                     const int32_t dims[4], double kappa, double mu,
                     const double phases[8], uint32_t flags, void *stream);
int wilson_dslash_eo_tm(const void *gauge, const void *in, void *out,
                        const int32_t dims[4], double kappa, double mu,
                        const double phases[8], int32_t out_parity,
                        uint32_t flags, void *stream);

/* Scratch bytes the solvers need for these dims and flags (0 on bad dims; 0
 * for WL_CANON with nrhs > 1, which the batched solvers do not take). With
 * WL_CANON (nrhs = 1) it includes the packed copies of the gauge field, b and
 * x. */
size_t wl_workspace_bytes(const int32_t dims[4], uint32_t flags, int32_t nrhs);

/* Solve M x = b (paper Sec. 4: the inversion S ~ M^-1 b) to
 * ||b - M x|| / ||b|| <= tol, the residual recomputed in FP64 on the full
 * lattice with the FP64 operator.
 *   solve_cg:       conjugate gradient on M^dag M x = M^dag b (CGNR);
 *   solve_bicgstab: BiCGStab on M.
 * With WL_EO both run on the Schur system Mhat_e x_e = b_e + kappa D_eo b_o and
 * reconstruct x_o = b_o + kappa D_oe x_e. With WL_MIXED the Krylov iterations
 * run in low precision -- FP32 (WL_F32 or no precision bits) or FP16 storage
 * with FP32 arithmetic (WL_F16S) -- on a copy of the links made at the start
 * of the solve, as one Krylov sequence with reliable updates: whenever the
 * low-precision residual norm has dropped by a factor delta since the last
 * update, the correction is added to the FP64 solution and the residual is
 * recomputed in FP64 and replaces the low-precision one. delta is 1e-4 (FP32
 * inner) or 0.2 (FP16) for CG, also updating when the residual has not halved
 * in 300 iterations, and 0.1 / 0.3 for BiCGStab (environment WL_DELTA_F32,
 * WL_DELTA_F16, WL_DELTA_BI_F32, WL_DELTA_BI_F16). A mixed BiCGStab whose
 * low-precision pass makes no progress continues in FP64 from its best
 * iterate (stats->fp64_iterations). FP64 is used for the solution, the
 * residuals, and the global reductions.
 * `gauge` is the packed FP64 gauge field (link format per flags); `b` and `x`
 * are packed FP64 full spinors; x is the initial guess with WL_X0, otherwise
 * it is overwritten from zero. With WL_CANON, `gauge` is the canonical
 * complex128 field U[V][4][3][3] and `b`, `x` canonical complex128 spinors
 * psi[V][4][3] (all device memory); the solve packs U (in the link format of
 * flags), b and, with WL_X0, x into its workspace, solves there, and unpacks
 * the solution into x -- the same result, bit for bit, as packing them
 * yourself. `work` is device scratch of at least
 * wl_workspace_bytes(dims, flags, 1) bytes. `stats` (host memory) may be NULL.
 * Blocks until the solve is complete. */
int solve_cg(const void *gauge, const void *b, void *x, const int32_t dims[4],
             double kappa, const double phases[8], double tol, int32_t maxiter,
             uint32_t flags, void *work, size_t work_bytes,
             wl_solve_stats *stats, void *stream);
int solve_bicgstab(const void *gauge, const void *b, void *x,
                   const int32_t dims[4], double kappa, const double phases[8],
                   double tol, int32_t maxiter, uint32_t flags, void *work,
                   size_t work_bytes, wl_solve_stats *stats, void *stream);

/* Solve M(mu) x = b for the twisted-mass operator above; everything else as
 * for solve_cg / solve_bicgstab (same flags, workspace size, statuses). With
 * WL_EO the Krylov iterations run on the Schur system
 * S_e x_e = b_e + kappa D_eo A^-1 b_o and x_o = A^-1 (b_o + kappa D_oe x_e);
 * acceptance is on ||b - M(mu) x|| / ||b|| in FP64. mu = 0 gives exactly
 * solve_cg / solve_bicgstab. */
int solve_cg_tm(const void *gauge, const void *b, void *x, const int32_t dims[4],
                double kappa, double mu, const double phases[8], double tol,
                int32_t maxiter, uint32_t flags, void *work, size_t work_bytes,
                wl_solve_stats *stats, void *stream);
int solve_bicgstab_tm(const void *gauge, const void *b, void *x,
                      const int32_t dims[4], double kappa, double mu,
                      const double phases[8], double tol, int32_t maxiter,
                      uint32_t flags, void *work, size_t work_bytes,
                      wl_solve_stats *stats, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation): solve_cg without a workspace argument.
 * The solver's scratch is a static device array of 64 MiB (64 << 20 bytes)
 * that the library holds on every GPU it runs on until the process ends;
 * this call allocates nothing (no hipMalloc/hipFree, no pinned host memory,
 * no autotuning events; status words are read through plain host memory).
 * Arguments, flags, layouts, results and return codes are those of
 * solve_cg, whose kernels it shares, so a solution has the bits of the same
 * solve_cg call. Returns WL_EWORKSPACE (nothing done) when
 * wl_workspace_bytes(dims, flags, 1) exceeds 64 MiB -- e.g. FP64 solves up to
 * about 32k sites (8^3 x 16 fits, 12^3 x 24 does not) -- and WL_EINVAL with
 * WL_GRAPH (graph instantiation allocates). Every call on one GPU uses that
 * GPU's one array and leaves its contents behind; the solver initialises
 * everything it reads, but calls that overlap in time on one GPU (from
 * several host threads) race on the array and must not be made. Blocks
 * until the solve is complete. */
int solve_cg_noalloc(const void *gauge, const void *b, void *x, const int32_t dims[4],
                     double kappa, const double phases[8], double tol, int32_t maxiter,
                     uint32_t flags, wl_solve_stats *stats, void *stream);

/* Batched operator: `in` and `out` each hold nrhs packed full spinors one
 * after another (stride wl_spinor_bytes(dims, flags, 2)); the modes are those
 * of wilson_dslash. All nrhs fields share the gauge field, whose links are
 * fetched from memory once per site and reused from cache for the others
 * (paper Sec. 4: the 12 spin-colour point sources of one propagator).
 * Asynchronous on `stream`; in and out must not overlap. */
int wilson_dslash_batch(const void *gauge, const void *in, void *out, int32_t nrhs,
                        const int32_t dims[4], double kappa, const double phases[8],
                        uint32_t flags, void *stream);

/* Batched CGNR: solve M x_r = b_r for 1 <= nrhs <= 64 right-hand sides on one
 * gauge field together. b and x each hold nrhs packed FP64 full spinors one
 * after another; flags as for solve_cg (WL_EO, WL_LINK12, WL_X0, WL_GRAPH, and
 * WL_MIXED with an FP32 or FP16-storage inner solve). Each RHS has its own
 * Krylov scalars, stops at its own tolerance and is restarted on its own FP64
 * true residual; with WL_MIXED each RHS runs the reliable-update sequence of
 * solve_cg, the FP64 replacements of all RHS together, so every solution has
 * the bits of the same RHS solved alone. `stats` (host, may be NULL) receives
 * nrhs entries. `work` needs
 * wl_workspace_bytes(dims, flags, nrhs) bytes. Returns WL_OK when every RHS
 * met tol, else a non-OK status of some RHS (see stats). Blocks until done. */
int solve_cg_batch(const void *gauge, const void *b, void *x, int32_t nrhs,
                   const int32_t dims[4], double kappa, const double phases[8],
                   double tol, int32_t maxiter, uint32_t flags, void *work,
                   size_t work_bytes, wl_solve_stats *stats, void *stream);

/* One problem of an uneven batch: its own lattice, kappa and gauge field. */
typedef struct {
    int32_t dims[4];      /* lattice extents (even, >= 2) */
    double kappa;         /* hopping parameter of this problem */
    const void *gauge;    /* packed FP64 gauge field (link format of flags) */
    const void *b;        /* packed FP64 full source spinor */
    void *x;              /* packed FP64 full solution (initial guess, WL_X0) */
} wl_problem;

/* Scratch bytes for solve_cg_problems on these problems (0 on bad dims). */
size_t wl_problems_workspace_bytes(const wl_problem *p, int32_t n, uint32_t flags);

/* Uneven batch: solve M_i x_i = b_i by CGNR for n independent problems of
 * any mix of lattice sizes, kappas and gauge fields (paper Sec. 4: inversions
 * for many configurations). Problems of one size are solved together as one
 * batched solve (each with its own gauge field and kappa; up to 64 per group),
 * and the groups run concurrently on library-owned streams. flags as for
 * solve_cg_batch (WL_EO, WL_LINK12, WL_X0, WL_GRAPH, WL_MIXED). The call waits for
 * `stream` to drain, then blocks until every problem is done; stats (host,
 * may be NULL) receives n entries in the order of p. Returns WL_OK when every
 * problem met tol, else a non-OK status of some problem. */
int solve_cg_problems(const wl_problem *p, int32_t n, const double phases[8], double tol,
                      int32_t maxiter, uint32_t flags, void *work, size_t work_bytes,
                      wl_solve_stats *stats, void *stream);

/* Meson correlators of one point-source propagator (paper Sec. 4, Eq. 1):
 *   C_Gamma(t) = - sum_xvec Tr( S^dag(x) g5 Gamma S(x) Gamma g5 ),  x = (xvec, t),
 * where the columns of the 12 x 12 spin-colour matrix S(x) are the 12
 * solutions of M x = b for the point sources of spin b and colour c at one
 * site (e.g. the result of solve_cg_batch on those sources): `props` holds
 * the 12 packed FP64 full spinors one after another (stride
 * wl_spinor_bytes(dims, WL_F64, 2)), field 3 b + c. The trace runs over spin
 * and colour, the 16 Gamma_n = g_x^n0 g_y^n1 g_z^n2 g_t^n3 (bits n0..n3 of
 * n; Gamma_15 = g5, Gamma_0 = 1) are those of the chiral basis, and t is
 * counted from the source's time slice t0 (0 <= t0 < Lt). `corr` (device)
 * receives double[16][Lt][2] (real, imaginary parts). Sums run in a fixed
 * order (bitwise reproducible). `work` is device scratch of
 * wl_meson_workspace_bytes(dims) bytes. Asynchronous on `stream`. */
size_t wl_meson_workspace_bytes(const int32_t dims[4]);
int wl_meson_correlators(const void *props, const int32_t dims[4], int32_t t0,
                         double *corr, void *work, size_t work_bytes, void *stream);

/* Pure gauge theory (paper Sec. 3: the SU(3) heatbath of the pure-gauge side,
 * after Creutz), on the CANONICAL complex128 gauge field U[V][4][3][3] on the
 * device (the layout wl_pack_gauge reads), with the Wilson plaquette action
 *   S = beta sum_P (1 - Re Tr U_P / 3).
 * wl_heatbath: nsweeps heat-bath sweeps in place. A sweep updates, for
 * mu = 0..3, the links of direction mu on the even and then the odd sites;
 * each link gets the Cabibbo-Marinari update over its SU(2) subgroups on
 * rows/columns (0,1), (1,2), (0,2), whose SU(2) heat-bath component x0 is
 * drawn by rejection (Kennedy-Pendleton for alpha = 2 beta |b| / 3 >= 1, the
 * unit disk's first coordinate below; at most 128 attempts, each accepted
 * with probability >= 0.41; a subgroup without an accepted draw keeps its
 * link). Random numbers: Philox4x32-10 with key (seed, 0x68656174) and
 * counter (site, mu + 4 subgroup + 16 attempt, sweep number, draw), sweep
 * numbers sweep0, sweep0 + 1, ...; the result does not depend on the launch
 * or on other work. Asynchronous on `stream`.
 * wl_plaquette: the mean plaquette sum_x sum_{mu<nu} Re Tr U_mu nu(x) / (18 V)
 * into *out (device double), through wl_plaquette_workspace_bytes(dims) of
 * work; fixed-order sums (bitwise reproducible). Asynchronous on `stream`. */
int wl_heatbath(void *gauge, const int32_t dims[4], double beta, int32_t nsweeps,
                uint32_t sweep0, uint32_t seed, void *stream);
size_t wl_plaquette_workspace_bytes(const int32_t dims[4]);
int wl_plaquette(const void *gauge, const int32_t dims[4], double *out, void *work,
                 size_t work_bytes, void *stream);

/* The same two on the PACKED FP64 18-real gauge field (what wl_pack_gauge
 * writes with WL_F64 and 18-real links, wl_gauge_bytes(dims, WL_F64) bytes),
 * whose loads are coalesced: wl_heatbath_packed performs the same
 * arithmetic on the same links and draws as wl_heatbath, so packing the
 * canonical field after wl_heatbath gives bitwise the field wl_heatbath_packed
 * leaves; the solvers take that field as it is, so a chain of configurations
 * needs no packing between the update and the measurement. wl_plaquette_packed
 * sums the sites in checkerboard order (the last bits may differ from
 * wl_plaquette). Same arguments, errors and asynchrony as above. */
int wl_heatbath_packed(void *gauge, const int32_t dims[4], double beta, int32_t nsweeps,
                       uint32_t sweep0, uint32_t seed, void *stream);
int wl_plaquette_packed(const void *gauge, const int32_t dims[4], double *out, void *work,
                        size_t work_bytes, void *stream);

/* Streaming device-to-device copy of `bytes` bytes (both pointers 16-byte
 * aligned, bytes a multiple of 16; the buffers must not overlap), loads then
 * non-temporal stores, 64 bytes per thread: the achievable-bandwidth
 * reference the operator kernels are measured against. Asynchronous on
 * `stream`. WL_EINVAL on misaligned or overlapping arguments. */
int wl_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Autotuning record. Batched operator launches (wilson_dslash_batch and the
 * batched solves) give each thread several right-hand sides at once, so one
 * link load serves all of them; the first launch of each shape (precision,
 * link format, operator, batch size, lattice) times every candidate count on
 * its own buffers and keeps the fastest (environment: WL_TUNE=0 disables
 * tuning, WL_TUNE_FILE=path keeps the choices in that file across processes).
 * Copies the record, one line per shape with the chosen count and the time of
 * each candidate, into buf (at most len - 1 bytes and a NUL; buf may be NULL)
 * and returns its full length. */
size_t wl_tuning_report(char *buf, size_t len);

/* ---------------------------------------------------------------------------
 * Serving: a solve server that admits requests as device memory and solve
 * slots free up, and runs the admitted solves concurrently (paper Sec. 4: many
 * inversions per gauge configuration, here served as a request stream).
 *
 * The server owns one device arena of `hbm_budget` bytes, taken at creation,
 * from which each admitted request's solver workspace (wl_workspace_bytes of
 * its lattice and the server's flags) is carved; gauge fields, sources and
 * solutions stay caller-owned device memory (gauge fields are typically kept
 * resident and shared by many requests) and must stay valid until the request
 * is collected. Requests are admitted earliest deadline first, the deadline
 * of a request being its submission time plus `site_slack` seconds per site
 * of its lattice (site_slack = 0: first-in first-out): that request starts as
 * soon as a slot is idle and its workspace fits in the free arena, and the
 * requests behind it wait until then. A positive site_slack lets small
 * lattices overtake large ones submitted at most site_slack * (V_large -
 * V_small) seconds earlier, so a large request is passed over for a bounded
 * time. Each slot is a host thread with its own stream, so the solves of all
 * admitted requests overlap on the device. With `merge` > 1 the slot also
 * takes up to merge - 1 further waiting requests of the same lattice size, if
 * that lattice has at most 131072 sites (a larger solve fills the device by
 * itself), oldest first, passing over other sizes, while the batch's workspace fits,
 * and solves them as one batched CG (each with its own gauge field, kappa,
 * source and solution; they are admitted and finish together). A request's
 * result does not depend on what else is running or on its batch mates
 * (every reduction has a fixed order): it is bitwise its solo solve.
 * ------------------------------------------------------------------------- */
typedef struct wl_server wl_server;   /* opaque */

typedef struct {
    size_t hbm_budget;    /* arena bytes for request workspaces (> 0)           */
    int32_t slots;        /* concurrent solves, 1..64                           */
    uint32_t flags;       /* solve_cg flags of every request (WL_EO, WL_MIXED,  */
                          /* WL_F32 / WL_F16S, WL_LINK12, WL_X0, WL_GRAPH)      */
    double tol;           /* relative true-residual target                       */
    int32_t maxiter;      /* iteration limit per request                         */
    double phases[8];     /* boundary phases, as for wilson_dslash               */
    int32_t merge;        /* most requests of one size solved as one batch,    */
                          /* 0..64 (0 or 1: every request alone)                */
    double site_slack;    /* admission deadline = submission + site_slack * V  */
                          /* seconds, V the lattice's sites; >= 0 (0: FIFO)     */
} wl_server_config;

/* Timestamps of one request, seconds since the server was created. */
typedef struct {
    double submitted;     /* wl_server_submit returned                          */
    double admitted;      /* a slot and its workspace were taken                 */
    double finished;      /* the solution is in x and the slot is free           */
} wl_request_times;

/* Create a server on the current device. Returns WL_OK and sets *out, or
 * WL_EINVAL (bad config), WL_EHIP (the arena could not be allocated). */
int wl_server_create(const wl_server_config *cfg, wl_server **out);

/* Queue a solve of M x = b for one problem (dims, kappa, packed FP64 gauge,
 * b and x as in wl_problem). Non-blocking; *ticket identifies the request
 * (a server numbers its tickets 1, 2, 3, ... in submission order).
 * WL_EINVAL for a bad problem, WL_EWORKSPACE when its workspace exceeds the
 * whole arena (it could never be admitted). */
int wl_server_submit(wl_server *srv, const wl_problem *p, uint64_t *ticket);

/* Block until request `ticket` finishes, collect it and return its solver
 * status (WL_OK when it met tol); stats and times may be NULL. WL_EINVAL for
 * an unknown or already collected ticket. */
int wl_server_wait(wl_server *srv, uint64_t ticket, wl_solve_stats *stats,
                   wl_request_times *times);

/* Block until any uncollected request finishes (oldest finished first),
 * collect it, set *ticket and return its status. WL_EINVAL when no request is
 * pending. */
int wl_server_next(wl_server *srv, uint64_t *ticket, wl_solve_stats *stats,
                   wl_request_times *times);

/* Requests submitted but not yet collected (queued, running or finished). */
int32_t wl_server_pending(wl_server *srv);

/* Finish every queued and running request, then release the slots, streams
 * and arena. Uncollected results are dropped (solutions are still in x). No
 * other call on srv may be in progress or follow. */
int wl_server_destroy(wl_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* WILSON_H */
