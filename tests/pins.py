"""Pins of the CPU oracle: facts fixed by the mathematics and the physics.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with the fact. None of them re-types the oracle's stencil:
they use closed forms (free-field plane waves), invariants (gamma5
hermiticity, gauge covariance), a differently assembled dense operator, and
library routines (LAPACK) or a different algorithm (Neumann series) for the
solves. ``tests/test_oracle_mutants.py`` plants mistakes in copies of the
oracle and checks that these pins catch each one.
"""
import itertools

import numpy as np

from paper_1112_5280_amd import synth
from tests.dense_ref import dense_dslash, parity_index

AP = np.array([1, 1, 1, -1], dtype=np.complex128)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) /
                 max(np.linalg.norm(np.asarray(b)), 1e-300))


def gammas(orc):
    return [orc.gamma(mu) for mu in range(4)]


# ---------------------------------------------------------------------------
def pin_gamma_algebra(orc):
    """Euclidean Clifford algebra, hermiticity, and the chiral gamma_5."""
    g = gammas(orc)
    g5 = orc.gamma(4)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0), "gamma not Hermitian"
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3], atol=1e-15)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=1e-15)


# ---------------------------------------------------------------------------
def _momenta(dims, phases):
    theta = np.angle(np.asarray(phases, dtype=np.complex128))
    return [[(2 * np.pi * n + theta[mu]) / dims[mu] for n in range(dims[mu])]
            for mu in range(4)]


def _plane_wave(dims, p):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                             np.arange(lx), indexing="ij")
    ph = p[0] * x + p[1] * y + p[2] * z + p[3] * t
    return np.exp(1j * ph).reshape(-1)


def pin_free_field_plane_wave(orc, dims=(4, 6, 2, 8), kappa=0.13,
                              phases=(np.exp(0.3j), np.exp(-1.1j), 1.0, -1.0)):
    """Unit links: M e^{ipx} w = e^{ipx} A(p) w with
    A(p) = (1 - 2 kappa sum cos p) + 2 i kappa sum sin(p_mu) gamma_mu, where the
    momenta satisfy p_mu L_mu = theta_mu mod 2 pi (twisted boundaries).
    Also checks that A's eigenvalues are 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p).
    """
    g = gammas(orc)
    U = synth.gauge_unit(dims)
    mom = _momenta(dims, phases)
    rng = np.random.default_rng(5)
    picks = [tuple(rng.integers(0, dims[mu]) for mu in range(4)) for _ in range(4)]
    picks.append((0, 0, 0, 0))
    for n in picks:
        p = [mom[mu][n[mu]] for mu in range(4)]
        A = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) + \
            2j * kappa * sum(np.sin(p[mu]) * g[mu] for mu in range(4))
        wave = _plane_wave(dims, p)
        w = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = wave[:, None, None] * w[None]
        out = orc.mop(U, psi, dims, kappa, phases)
        expect = wave[:, None, None] * (A @ w)[None]
        assert rel(out, expect) < 1e-13, "plane wave not mapped by A(p)"
        s = np.sqrt(sum(np.sin(x) ** 2 for x in p))
        lam = np.linalg.eigvals(A)
        c = 1 - 2 * kappa * sum(np.cos(p))
        want = np.array([c - 2j * kappa * s] * 2 + [c + 2j * kappa * s] * 2)
        assert _sorted_close(lam, want, 1e-13)


def _dense_from_apply(apply, n):
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1
        cols.append(apply(e))
    return np.stack(cols, axis=1)


def _sorted_close(a, b, tol):
    ka = np.lexsort((np.round(a.imag, 6), np.round(a.real, 6)))
    kb = np.lexsort((np.round(b.imag, 6), np.round(b.real, 6)))
    return np.max(np.abs(a[ka] - b[kb])) < tol


def pin_free_field_spectrum(orc, dims=(2, 4, 2, 4), kappa=0.13):
    """All 12V eigenvalues of M on unit links with antiperiodic time equal the
    closed form 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p), each 6-fold, with
    p_t = (2n+1) pi / L_t."""
    V = int(np.prod(dims))
    U = synth.gauge_unit(dims)
    M = _dense_from_apply(
        lambda e: orc.mop(U, e.reshape(V, 4, 3), dims, kappa, AP).reshape(-1),
        12 * V)
    ev = np.linalg.eigvals(M)
    mom = _momenta(dims, AP)
    want = []
    for n in itertools.product(*[range(d) for d in dims]):
        p = [mom[mu][n[mu]] for mu in range(4)]
        c = 1 - 2 * kappa * sum(np.cos(p))
        s = np.sqrt(sum(np.sin(x) ** 2 for x in p))
        want += [c + 2j * kappa * s] * 6 + [c - 2j * kappa * s] * 6
    assert _sorted_close(ev, np.array(want), 1e-10), "free-field spectrum"


# ---------------------------------------------------------------------------
def pin_dense_kron(orc, dims=(2, 4, 2, 4), seed=11, kappa=0.11):
    """The oracle's D_W, M and their adjoints equal a dense operator assembled
    independently from Kronecker blocks (extent-2 neighbours coincide)."""
    V = int(np.prod(dims))
    U = synth.gauge_haar(dims, seed)
    phases = np.exp(1j * np.array([0.4, -0.9, 2.1, np.pi]))
    D = dense_dslash(U, dims, gammas(orc), phases)
    psi = synth.gaussian_spinor(dims, seed + 1)
    v = psi.reshape(-1)
    assert rel(orc.dslash(U, psi, dims, phases).reshape(-1), D @ v) < 1e-13
    assert rel(orc.dslash(U, psi, dims, phases, dagger=True).reshape(-1),
               D.conj().T @ v) < 1e-13
    M = np.eye(12 * V) - kappa * D
    assert rel(orc.mop(U, psi, dims, kappa, phases).reshape(-1), M @ v) < 1e-13
    assert rel(orc.mop(U, psi, dims, kappa, phases, dagger=True).reshape(-1),
               M.conj().T @ v) < 1e-13


def pin_gamma5_hermiticity(orc, dims=(4, 4, 4, 4), kappa=0.12):
    """<phi, M psi> = <g5 M g5 phi, psi> on a Haar field (Eq. 1 relies on it)."""
    U = synth.gauge_haar(dims, 3)
    phi = synth.gaussian_spinor(dims, 4)
    psi = synth.gaussian_spinor(dims, 5)
    lhs = np.vdot(phi, orc.mop(U, psi, dims, kappa))
    rhs = np.vdot(orc.mop(U, phi, dims, kappa, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs), "gamma5 hermiticity"
    # and D_W itself
    lhs = np.vdot(phi, orc.dslash(U, psi, dims))
    rhs = np.vdot(orc.dslash(U, phi, dims, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def gauge_transform(U, dims, omega):
    """U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dagger."""
    V = int(np.prod(dims))
    out = np.empty_like(U)
    x, y, z, t = synth.site_coords(dims, np.arange(V))
    c = [x, y, z, t]
    for mu in range(4):
        cf = list(c)
        cf[mu] = (c[mu] + 1) % dims[mu]
        sf = synth.site_index(dims, *cf)
        out[:, mu] = omega @ U[:, mu] @ np.conj(np.swapaxes(omega[sf], 1, 2))
    return out


def pin_gauge_covariance(orc, dims=(4, 4, 2, 6), kappa=0.12):
    """M[U^Omega](Omega psi) = Omega M[U] psi for random local SU(3) Omega."""
    V = int(np.prod(dims))
    U = synth.gauge_haar(dims, 7)
    omega = synth.haar_su3(V, np.random.default_rng(8))
    psi = synth.gaussian_spinor(dims, 9)
    Ug = gauge_transform(U, dims, omega)
    psig = np.einsum("sab,sib->sia", omega, psi)
    lhs = orc.mop(Ug, psig, dims, kappa)
    rhs = np.einsum("sab,sib->sia", omega, orc.mop(U, psi, dims, kappa))
    assert rel(lhs, rhs) < 1e-13, "gauge covariance"


# ---------------------------------------------------------------------------
def pin_eo_split(orc, dims=(4, 2, 6, 4)):
    """D_W = D_eo + D_oe; each block sees only the other parity's input."""
    U = synth.gauge_haar(dims, 13)
    psi = synth.gaussian_spinor(dims, 14)
    from oracle import parity_mask
    odd = parity_mask(dims)
    for dag in (False, True):
        full = orc.dslash(U, psi, dims, dagger=dag)
        e = orc.dslash_eo(U, psi, dims, 0, dagger=dag)
        o = orc.dslash_eo(U, psi, dims, 1, dagger=dag)
        assert rel(e + o, full) < 1e-14
        assert np.all(e[odd] == 0) and np.all(o[~odd] == 0)
        junk = psi.copy()
        junk[~odd] = 7.0  # even input must not enter D_{even,odd}
        assert rel(orc.dslash_eo(U, junk, dims, 0, dagger=dag), e) < 1e-14


def pin_schur_dense(orc, dims=(2, 4, 2, 4), kappa=0.13):
    """Mhat = M_ee - M_eo M_oo^-1 M_oe by dense block elimination (and its
    adjoint for the dagger), on both parities."""
    U = synth.gauge_haar(dims, 15)
    V = int(np.prod(dims))
    D = dense_dslash(U, dims, gammas(orc), AP)
    M = np.eye(12 * V) - kappa * D
    ev, od = parity_index(dims)
    psi = synth.gaussian_spinor(dims, 16)
    for par, (a, b) in ((0, (ev, od)), (1, (od, ev))):
        S = M[np.ix_(a, a)] - M[np.ix_(a, b)] @ np.linalg.solve(
            M[np.ix_(b, b)], M[np.ix_(b, a)])
        v = np.zeros(12 * V, dtype=np.complex128)
        v[a] = psi.reshape(-1)[a]
        for dag in (False, True):
            out = orc.schur(U, v.reshape(V, 4, 3), dims, kappa, par,
                            dagger=dag).reshape(-1)
            want = (S.conj().T if dag else S) @ v[a]
            assert rel(out[a], want) < 1e-13
            assert np.all(out[b] == 0)


def pin_sites(orc, dims=(4, 4, 2, 6), kappa=0.14):
    """The site-sampled operators agree with the whole-lattice ones."""
    U = synth.gauge_haar(dims, 17)
    psi = synth.gaussian_spinor(dims, 18)
    sites = np.random.default_rng(19).choice(synth.volume(dims), 37,
                                             replace=False)
    for dag in (False, True):
        assert rel(orc.mop_sites(U, psi, dims, kappa, sites, dagger=dag),
                   orc.mop(U, psi, dims, kappa, dagger=dag)[sites]) < 1e-15
        assert rel(orc.dslash_sites(U, psi, dims, sites, dagger=dag),
                   orc.dslash(U, psi, dims, dagger=dag)[sites]) < 1e-15


# ---------------------------------------------------------------------------
def pin_solvers_lapack(orc, dims=(4, 4, 4, 4), kappa=0.12, maxiter=3000):
    """CGNR and BiCGStab reach the LAPACK solution of the dense system."""
    U = synth.gauge_haar(dims, 0)
    b = synth.gaussian_spinor(dims, 1)
    V = int(np.prod(dims))
    D = dense_dslash(U, dims, gammas(orc), AP)
    M = np.eye(12 * V) - kappa * D
    xs = np.linalg.solve(M, b.reshape(-1))
    # ||D_W|| <= 8 for unitary links and unit phases, so for kappa < 1/8
    # cond(M) <= (1 + 8 kappa) / (1 - 8 kappa)
    cond = (1 + 8 * kappa) / (1 - 8 * kappa)
    # CG on M^dag M contracts the error by (c - 1)/(c + 1) per step with
    # c = cond(M), so ln(2/tol) c / 2 steps suffice; on so well-conditioned a
    # system the recursive residual tracks the true one to rounding, so a
    # correct method needs at most a couple of true-residual restarts.
    it_bound = cond * np.log(2 / 1e-10) / 2
    for solver in (orc.cgnr, orc.cgnr_eo, orc.bicgstab):
        x, st = solver(U, b, dims, kappa, tol=1e-10, maxiter=maxiter)
        assert st["status"] == 0, st
        res = np.linalg.norm(b.reshape(-1) - M @ x.reshape(-1)) / np.linalg.norm(b)
        assert res <= 1e-10, res
        assert rel(x.reshape(-1), xs) <= cond * 1e-10
        assert st["restarts"] <= 2 and st["iterations"] <= it_bound, st


def pin_neumann(orc, dims=(4, 4, 2, 4), kappa=0.12):
    """For kappa < 1/8, x = sum_k (kappa D_W)^k b (a different algorithm)."""
    U = synth.gauge_haar(dims, 21)
    b = synth.gaussian_spinor(dims, 22)
    term = b.copy()
    x = b.copy()
    for _ in range(2000):
        term = kappa * orc.dslash(U, term, dims)
        x = x + term
        if np.linalg.norm(term) < 1e-15 * np.linalg.norm(b):
            break
    xc, st = orc.cgnr(U, b, dims, kappa, tol=1e-12, maxiter=3000)
    assert st["status"] == 0
    assert rel(xc, x) < 1e-10


def pin_free_field_solve(orc, dims=(4, 2, 4, 8), kappa=0.12):
    """Unit links: the source e^{ipx} w, w an eigenvector of A(p), has the
    solution e^{ipx} w / lambda."""
    g = gammas(orc)
    U = synth.gauge_unit(dims)
    mom = _momenta(dims, AP)
    p = [mom[0][1], mom[1][1], mom[2][3], mom[3][2]]
    A = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) + \
        2j * kappa * sum(np.sin(p[mu]) * g[mu] for mu in range(4))
    lam, vec = np.linalg.eig(A)
    w = np.outer(vec[:, 0], np.array([0.3, -1.0j, 0.7]))
    b = _plane_wave(dims, p)[:, None, None] * w[None]
    for solver in (orc.cgnr, orc.cgnr_eo, orc.bicgstab):
        x, st = solver(U, b, dims, kappa, tol=1e-12, maxiter=3000)
        assert st["status"] == 0
        assert rel(x, b / lam[0]) < 1e-10


def pin_eo_solve_odd_rows(orc, dims=(4, 2, 4, 6), kappa=0.13):
    """The even-odd solve fixes x_o from x_e through the odd rows of M x = b,
    so those rows hold to rounding whatever x_e is; and its solution agrees
    with LAPACK's dense solve of the full system within cond * tol."""
    U = synth.gauge_smooth(dims, 0.3, 31)
    b = synth.gaussian_spinor(dims, 32)
    V = int(np.prod(dims))
    _, odd = parity_index(dims)
    for tol, maxiter in ((1e-2, 3000), (1e-12, 3000)):
        x, st = orc.cgnr_eo(U, b, dims, kappa, tol=tol, maxiter=maxiter)
        r = (b - orc.mop(U, x, dims, kappa)).reshape(-1)
        assert np.linalg.norm(r[odd]) <= 1e-14 * np.linalg.norm(b), tol
        assert st["status"] == 0 and st["true_res"] <= tol, st
    D = dense_dslash(U, dims, gammas(orc), AP)
    M = np.eye(12 * V) - kappa * D
    xs = np.linalg.solve(M, b.reshape(-1))
    assert rel(x.reshape(-1), xs) <= np.linalg.cond(M) * 2e-12


def _g5_dense(orc, V):
    """gamma_5 = gamma_x gamma_y gamma_z gamma_t on every site and colour."""
    g = gammas(orc)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return np.kron(np.eye(V), np.kron(g5, np.eye(3)))


def pin_tm_free_field_spectrum(orc, dims=(2, 4, 2, 4), kappa=0.13, mu=0.37):
    """Unit links: the 12V eigenvalues of M(mu) = 1 + 2ik mu g5 - k D_W are
    1 - 2k sum cos p +- 2ik sqrt(mu^2 + sum sin^2 p), each 6-fold (g5
    anticommutes with every gamma_mu, so (mu g5 + sum sin p gamma)^2 is
    mu^2 + sum sin^2 p)."""
    V = int(np.prod(dims))
    U = synth.gauge_unit(dims)
    M = _dense_from_apply(
        lambda e: orc.mop_tm(U, e.reshape(V, 4, 3), dims, kappa, mu, AP).reshape(-1),
        12 * V)
    ev = np.linalg.eigvals(M)
    mom = _momenta(dims, AP)
    want = []
    for n in itertools.product(*[range(d) for d in dims]):
        p = [mom[m][n[m]] for m in range(4)]
        c = 1 - 2 * kappa * sum(np.cos(p))
        s2 = np.sqrt(mu * mu + sum(np.sin(x) ** 2 for x in p))
        want += [c + 2j * kappa * s2] * 6 + [c - 2j * kappa * s2] * 6
    assert _sorted_close(ev, np.array(want), 1e-10), "twisted free-field spectrum"


def pin_tm_dense_and_adjoint(orc, dims=(2, 4, 2, 4), seed=41, kappa=0.12, mu=0.21):
    """M(mu) equals the dense Kronecker-assembled 1 - k D_W + 2ik mu g5, its
    adjoint is the conjugate transpose, g5 M(mu) g5 = M(-mu)^dag, and mu = 0 is
    the Wilson operator."""
    V = int(np.prod(dims))
    U = synth.gauge_haar(dims, seed)
    D = dense_dslash(U, dims, gammas(orc), AP)
    G5 = _g5_dense(orc, V)
    M = np.eye(12 * V) - kappa * D + 2j * kappa * mu * G5
    psi = synth.gaussian_spinor(dims, seed + 1)
    v = psi.reshape(-1)
    assert rel(orc.mop_tm(U, psi, dims, kappa, mu).reshape(-1), M @ v) < 1e-13
    assert rel(orc.mop_tm(U, psi, dims, kappa, mu, dagger=True).reshape(-1),
               M.conj().T @ v) < 1e-13
    g5m = (G5 @ orc.mop_tm(U, (G5 @ v).reshape(V, 4, 3), dims, kappa, -mu).reshape(-1))
    assert rel(g5m, orc.mop_tm(U, psi, dims, kappa, mu, dagger=True).reshape(-1)) < 1e-13
    assert rel(orc.mop_tm(U, psi, dims, kappa, 0.0), orc.mop(U, psi, dims, kappa)) < 1e-15


def pin_tm_schur_block_elimination(orc, dims=(4, 2, 4, 6), kappa=0.13, mu=0.27):
    """Block elimination of M(mu) on parity p: for psi supported on parity p and
    x = psi + kappa A^-1 D_{1-p,p} psi (A = 1 + 2ik mu g5, inverted by LAPACK on
    the dense site-diagonal matrix), M(mu) x equals S_p psi on parity p and
    vanishes on parity 1-p; the adjoint is the conjugate transpose."""
    V = int(np.prod(dims))
    U = synth.gauge_haar(dims, 45)
    G5 = _g5_dense(orc, V)
    Ainv = np.linalg.inv(np.eye(12 * V) + 2j * kappa * mu * G5)
    par = np.repeat(parity_index_sites(dims), 12)
    for p in (0, 1):
        psi = synth.gaussian_spinor(dims, 46 + p) * (parity_index_sites(dims) == p)[:, None, None]
        d = orc.dslash_eo(U, psi, dims, 1 - p).reshape(-1)
        x = psi.reshape(-1) + kappa * (Ainv @ d)
        mx = orc.mop_tm(U, x.reshape(V, 4, 3), dims, kappa, mu).reshape(-1)
        s = orc.schur_tm(U, psi, dims, kappa, mu, p).reshape(-1)
        assert rel(mx[par == p], s[par == p]) < 1e-13
        assert np.linalg.norm(mx[par != p]) < 1e-13 * np.linalg.norm(s)
        assert not s[par != p].any()
        phi = synth.gaussian_spinor(dims, 50 + p) * (parity_index_sites(dims) == p)[:, None, None]
        lhs = np.vdot(phi, orc.schur_tm(U, psi, dims, kappa, mu, p))
        rhs = np.vdot(orc.schur_tm(U, phi, dims, kappa, mu, p, dagger=True), psi)
        assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    assert rel(orc.schur_tm(U, psi, dims, kappa, 0.0, 1), orc.schur(U, psi, dims, kappa, 1)) < 1e-15


def parity_index_sites(dims):
    """Parity (x+y+z+t) mod 2 of every site, canonical order."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return ((x + y + z + t) % 2).reshape(-1)


def pin_tm_solve_lapack(orc, dims=(2, 4, 2, 4), kappa=0.12, mu=0.15):
    """CGNR on M(mu) reaches LAPACK's solution of the dense twisted system."""
    V = int(np.prod(dims))
    U = synth.gauge_haar(dims, 43)
    b = synth.gaussian_spinor(dims, 44)
    M = np.eye(12 * V) - kappa * dense_dslash(U, dims, gammas(orc), AP) + \
        2j * kappa * mu * _g5_dense(orc, V)
    xs = np.linalg.solve(M, b.reshape(-1))
    x, st = orc.cgnr_tm(U, b, dims, kappa, mu, tol=1e-11, maxiter=3000)
    assert st["status"] == 0, st
    assert rel(x.reshape(-1), xs) <= np.linalg.cond(M) * 2e-11
    assert abs(orc.true_residual_tm(U, b, x, dims, kappa, mu) - st["true_res"]) < 1e-13


def _random_props(dims, seed):
    V = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    return rng.standard_normal((12, V, 4, 3)) + 1j * rng.standard_normal((12, V, 4, 3))


def _site_matrix(props):
    """S[x][i][j]: sink (spin, colour) i, source j = 3 b + c."""
    V = props.shape[1]
    return np.transpose(props.reshape(12, V, 12), (1, 2, 0))


def pin_meson_pion_and_completeness(orc, dims=(2, 4, 2, 6)):
    """Eq. 1 with Gamma = g5 is -sum |S|^2 per time slice; over the 16 Gammas,
    sum_n Gamma_n^2 C_n = -4 sum_colours |Tr_spin S|^2 (the completeness of the
    Dirac basis: sum_n Gamma_n X Gamma_n^-1 = 4 Tr(X) for 4 x 4 X, with
    Gamma_n^-1 = Gamma_n^2 Gamma_n, Gamma_n^2 = +-1); t is counted from t0."""
    g = gammas(orc)
    V = int(np.prod(dims))
    props = _random_props(dims, 61)
    S = _site_matrix(props)
    t_of = np.repeat(np.arange(dims[3]), V // dims[3])
    for t0 in (0, 3):
        C = orc.meson(props, dims, t0)
        pion = np.zeros(dims[3])
        comp = np.zeros(dims[3])
        trs = np.einsum("xaiaj->xij", S.reshape(V, 4, 3, 4, 3))
        for x in range(V):
            tr = (t_of[x] - t0) % dims[3]
            pion[tr] += np.sum(np.abs(S[x]) ** 2)
            comp[tr] += np.sum(np.abs(trs[x]) ** 2)
        assert rel(C[15], -pion) < 1e-13
        sq = []
        for n in range(16):
            m = np.eye(4)
            for mu in range(4):
                if n >> mu & 1:
                    m = m @ g[mu]
            sq.append((m @ m)[0, 0].real)
        assert rel(sum(sq[n] * C[n] for n in range(16)), -4 * comp) < 1e-13


def pin_meson_gauge_invariance(orc, dims=(2, 2, 4, 4)):
    """S(x) -> Omega(x) S(x) Omega(x0)^dag (colour rotations at sink and source)
    leaves every C_Gamma(t) unchanged."""
    V = int(np.prod(dims))
    props = _random_props(dims, 62)
    S = _site_matrix(props).reshape(V, 4, 3, 12)
    om = synth.haar_su3(V, np.random.default_rng(63))
    om0 = synth.haar_su3(1, np.random.default_rng(64))[0]
    S2 = np.einsum("xab,xsbj->xsaj", om, S)                 # sink colour
    S2 = S2.reshape(V, 12, 4, 3)
    S2 = np.einsum("xisb,cb->xisc", S2, om0.conj())         # source colour
    props2 = np.transpose(S2.reshape(V, 12, 12), (2, 0, 1)).reshape(12, V, 4, 3)
    assert rel(orc.meson(props2, dims), orc.meson(props, dims)) < 1e-13


def pin_meson_time_reversal(orc, dims=(2, 2, 2, 8), kappa=0.12):
    """On a time-reversal symmetric field (spatial links equal at t and -t,
    U_t(x, t) = U_t(x, -t-1)^dag; the antiperiodic wrap maps to itself) the
    point-source propagator from t = 0 obeys S(-t) = T S(t) T^-1 up to the
    source's transform, T = g_t g5 (it anticommutes with g_t, commutes with the
    spatial g_k), so every channel of Eq. 1 is even or odd in t:
    |C_Gamma(t)| = |C_Gamma(Lt - t)|, the pion (always negative) exactly even.
    The propagators are the oracle's own CGNR solves."""
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    base = synth.gauge_haar(dims, 81).reshape(Lt, Lz, Ly, Lx, 4, 3, 3)
    U = np.empty_like(base)
    for t in range(Lt):
        U[t, ..., :3, :, :] = base[min(t, Lt - t), ..., :3, :, :]
    for t in range(Lt // 2):
        U[t, ..., 3, :, :] = base[t, ..., 3, :, :]
        U[Lt - 1 - t, ..., 3, :, :] = np.conj(np.swapaxes(base[t, ..., 3, :, :], -1, -2))
    U = U.reshape(V, 4, 3, 3)
    mirror = [0] + list(range(Lt - 1, 0, -1))

    def correlators(field):
        props = np.empty((12, V, 4, 3), np.complex128)
        for j in range(12):
            x, st = orc.cgnr(field, synth.point_source(dims, 0, j // 3, j % 3), dims, kappa,
                             tol=1e-13)
            assert st["status"] == 0, st
            props[j] = x
        return orc.meson(props, dims, 0)

    C = correlators(U)
    assert (C[15].real < 0).all()
    assert np.abs(C[15] - C[15, mirror]).max() < 1e-10 * np.abs(C[15]).max()
    assert np.abs(np.abs(C) - np.abs(C[:, mirror])).max() < 1e-10 * np.abs(C).max()
    # the symmetry is the field's: the unsymmetrised field breaks it
    C0 = correlators(base.reshape(V, 4, 3, 3))
    assert np.abs(C0[15] - C0[15, mirror]).max() > 1e-3 * np.abs(C0[15]).max()


def pin_philox_known_answers(orc):
    """Philox4x32-10 reproduces the known-answer vectors published with the
    generator (Random123): zero counter and key, all-ones, and the digits of
    pi."""
    cases = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 4, (0xffffffff, 0xffffffff),
              (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for ctr, key, want in cases:
        assert tuple(orc.philox(ctr, key)) == want, (ctr, key)


def pin_kp_density(orc):
    """The heat bath's x0 draw samples the density proportional to
    sqrt(1 - x0^2) exp(alpha x0) on [-1, 1] (Kennedy-Pendleton for alpha >= 1,
    rejection from the unit disk's first coordinate below): every draw is
    accepted, the mean is I_2(alpha)/I_1(alpha), and a Kolmogorov-Smirnov test
    against the numerically integrated distribution function accepts it --
    at alpha = 0 (the semicircle), in the strong-coupling range where
    Kennedy-Pendleton alone is seldom accepted, and on both sides of the
    switch at alpha = 1."""
    from scipy import integrate, special, stats
    n = 200000
    x = orc.kp_samples(0.0, n, seed=5)
    assert (np.abs(x) <= 1).all()
    assert abs(x.mean()) < 5 * 0.5 / np.sqrt(n)
    for alpha in (0.05, 0.4, 0.99, 1.0, 2.5, 12.0):
        x = orc.kp_samples(alpha, n, seed=5)
        assert (np.abs(x) <= 1).all(), alpha
        mean = special.iv(2, alpha) / special.iv(1, alpha)
        z = integrate.quad(lambda t: np.sqrt(1 - t * t) * np.exp(alpha * t), -1, 1)[0]
        m2 = integrate.quad(lambda t: t * t * np.sqrt(1 - t * t) * np.exp(alpha * t), -1, 1)[0] / z
        assert abs(x.mean() - mean) < 5 * np.sqrt((m2 - mean ** 2) / n), (alpha, x.mean(), mean)
        grid = np.linspace(-1, 1, 200001)
        dens = np.sqrt(1 - grid * grid) * np.exp(alpha * grid)
        cum = np.concatenate([[0.0], np.cumsum((dens[1:] + dens[:-1]) / 2 * np.diff(grid))])
        cum /= cum[-1]
        assert stats.kstest(x[:20000], lambda q: np.interp(q, grid, cum)).pvalue > 1e-4, alpha


def pin_heatbath_unitary_and_strong_coupling(orc, dims=(4, 4, 4, 4)):
    """Heat-bath sweeps keep every link in SU(3); at strong coupling the mean
    plaquette is beta/18 to leading order (beta = 0.3: corrections are far
    below the statistical error), and at weak coupling it is 1 - 2/beta to
    leading order (equipartition over the 8 gauge degrees of freedom of each
    of the 3 non-gauge link directions per site, beta = 80)."""
    V = int(np.prod(dims))
    U = synth.gauge_haar(dims, 71)
    orc.heatbath(U, dims, 0.3, 20, sweep0=0, seed=9)
    m = U.reshape(-1, 3, 3)
    assert np.abs(m @ np.conj(np.swapaxes(m, 1, 2)) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(m) - 1).max() < 1e-13
    ps = []
    for k in range(60):
        orc.heatbath(U, dims, 0.3, 1, sweep0=20 + k, seed=9)
        ps.append(orc.plaquette(U, dims))
    p = float(np.mean(ps))
    err = float(np.std(ps)) / np.sqrt(len(ps))
    assert abs(p - 0.3 / 18) < 5 * err + 2e-4, (p, err)
    U = synth.gauge_unit(dims)
    orc.heatbath(U, dims, 80.0, 30, sweep0=0, seed=10)
    ps = []
    for k in range(30):
        orc.heatbath(U, dims, 80.0, 1, sweep0=30 + k, seed=10)
        ps.append(orc.plaquette(U, dims))
    assert abs(np.mean(ps) - (1 - 2 / 80.0)) < 2e-3, np.mean(ps)


def pin_plaquette(orc, dims=(4, 4, 2, 4)):
    """Unit links give plaquette 1; the plaquette is gauge invariant."""
    assert abs(orc.plaquette(synth.gauge_unit(dims), dims) - 1.0) < 1e-15
    V = int(np.prod(dims))
    U = synth.gauge_smooth(dims, 0.3, 23)
    omega = synth.haar_su3(V, np.random.default_rng(24))
    p0 = orc.plaquette(U, dims)
    p1 = orc.plaquette(gauge_transform(U, dims, omega), dims)
    assert abs(p0 - p1) < 1e-13


def pin_singular_extremes_dense(orc, dims=(2, 4, 2, 4), seed=25, kappa=0.13):
    """The Lanczos estimate of M's extreme singular values equals LAPACK's SVD
    of the dense operator on a Haar field."""
    V = int(np.prod(dims))
    U = synth.gauge_haar(dims, seed)
    M = _dense_from_apply(
        lambda e: orc.mop(U, e.reshape(V, 4, 3), dims, kappa, AP).reshape(-1),
        12 * V)
    sv = np.linalg.svd(M, compute_uv=False)
    smax, smin, cond = orc.singular_extremes(U, dims, kappa, steps=12 * V)
    assert abs(smax - sv[0]) <= 1e-10 * sv[0], (smax, sv[0])
    assert abs(smin - sv[-1]) <= 1e-8 * sv[-1], (smin, sv[-1])
    assert abs(cond - sv[0] / sv[-1]) <= 1e-8 * cond


def pin_singular_extremes_free_field(orc, dims=(4, 4, 4, 8), kappa=0.12):
    """Unit links: M is normal (a plane wave of momentum p spans an invariant
    space on which M acts as A(p)), so its singular values are the moduli
    |1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p)| over the lattice momenta."""
    U = synth.gauge_unit(dims)
    mom = _momenta(dims, AP)
    mods = []
    for n in itertools.product(*[range(d) for d in dims]):
        p = [mom[mu][n[mu]] for mu in range(4)]
        c = 1 - 2 * kappa * sum(np.cos(p))
        s = 2 * kappa * np.sqrt(sum(np.sin(x) ** 2 for x in p))
        mods.append(abs(c + 1j * s))
    smax, smin, cond = orc.singular_extremes(U, dims, kappa, steps=200)
    assert abs(smax - max(mods)) <= 1e-10 * max(mods), (smax, max(mods))
    assert abs(smin - min(mods)) <= 1e-10 * min(mods), (smin, min(mods))


ALL_PINS = [
    pin_gamma_algebra, pin_free_field_plane_wave, pin_free_field_spectrum,
    pin_dense_kron, pin_gamma5_hermiticity, pin_gauge_covariance,
    pin_eo_split, pin_schur_dense, pin_sites, pin_solvers_lapack,
    pin_neumann, pin_free_field_solve, pin_eo_solve_odd_rows, pin_plaquette,
    pin_tm_free_field_spectrum, pin_tm_dense_and_adjoint, pin_tm_solve_lapack,
    pin_tm_schur_block_elimination, pin_meson_pion_and_completeness,
    pin_meson_gauge_invariance, pin_meson_time_reversal, pin_philox_known_answers,
    pin_kp_density,
    pin_heatbath_unitary_and_strong_coupling,
    pin_singular_extremes_dense, pin_singular_extremes_free_field,
]
