"""Twisted-mass Wilson fermions (paper Sec. 3: the group's twisted-mass
action) on the GPU against the oracle: M(mu) = 1 + 2 i kappa mu g5 - kappa D_W,
its adjoint, the even-odd Schur complement S_p = A - kappa^2 D A^-1 D with
A = 1 + 2 i kappa mu g5, and the solves of M(mu) x = b (every solution checked
by the oracle's FP64 twisted residual). mu = 0 reproduces the Wilson calls
bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_5280_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (6, 4, 6, 10)]
PHASES = (1.0, np.exp(0.7j), 1.0, -1.0)


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("prec", [0x0, 0x1, 0x2], ids=["f64", "f32", "f16s"])
@pytest.mark.parametrize("link", [0x0, 0x4], ids=["link18", "link12"])
def test_twisted_operator(w, dims, prec, link):
    kappa, mu = 0.137, 0.31
    U = synth.gauge_smooth(dims, 0.3, 7)
    psi = synth.gaussian_spinor(dims, 8)
    G = w.pack_gauge(U, dims, prec | link)
    P = w.pack_spinor(psi, dims, prec)
    O = w.empty_spinor(dims, prec)
    for dag in (False, True):
        f = prec | link | (w.DAG if dag else 0)
        w.wilson_dslash_tm(G, P, O, dims, kappa, mu, PHASES, f)
        got = gu.to_np(w.unpack_spinor(O, dims, prec))
        want = oracle.mop_tm(U, psi, dims, kappa, mu, PHASES, dagger=dag)
        gu.assert_close(got, want, gu.TOL[prec], "M(mu) dag=%d" % dag)
    par = gu.parity_of_sites(dims)
    for p in (0, 1):
        sel = par == p
        psi_p = psi * sel[:, None, None]
        for dag in (False, True):
            f = prec | link | (w.DAG if dag else 0)
            full = w.empty_spinor(dims, prec, 2)
            w.wilson_dslash_eo_tm(G, w.parity_block(P, dims, prec, p), full, dims, kappa, mu, p,
                                  PHASES, f)
            got = gu.half_to_canon(w, w.parity_block(full, dims, prec, p), dims, prec, p)
            want = oracle.schur_tm(U, psi_p, dims, kappa, mu, p, PHASES, dagger=dag)
            gu.assert_close(got[sel], want[sel], gu.TOL[prec], "S_p p=%d dag=%d" % (p, dag))


def test_zero_twist_is_wilson_bitwise(w):
    dims, kappa = (6, 4, 6, 10), 0.13
    U = synth.gauge_haar(dims, 3)
    b = synth.gaussian_spinor(dims, 4)
    G = w.pack_gauge(U, dims)
    P = w.pack_spinor(b, dims)
    # zero-filled, so the padding entries the operators never touch are equal
    O1, O2 = w.zeros_spinor(dims), w.zeros_spinor(dims)
    for f in (0, w.DAG):
        w.wilson_dslash(G, P, O1, dims, kappa, flags=f)
        w.wilson_dslash_tm(G, P, O2, dims, kappa, 0.0, flags=f)
        gu.sync()
        assert torch.equal(O1, O2)
        w.wilson_dslash_eo(G, w.parity_block(P, dims, 0, 0), O1, dims, kappa, 0, flags=f)
        w.wilson_dslash_eo_tm(G, w.parity_block(P, dims, 0, 0), O2, dims, kappa, 0.0, 0, flags=f)
        gu.sync()
        assert torch.equal(O1, O2)
    X1, X2 = w.zeros_spinor(dims), w.zeros_spinor(dims)
    s1 = w.solve_cg(G, P, X1, dims, kappa, flags=w.EO)
    s2 = w.solve_cg_tm(G, P, X2, dims, kappa, 0.0, flags=w.EO)
    assert s1["iterations"] == s2["iterations"] and torch.equal(X1, X2)


TM_SOLVES = [("cg", 0x0), ("cg", 0x20), ("cg", 0x60), ("cg", 0x62), ("cg", 0x24),
             ("bicgstab", 0x20), ("bicgstab", 0x60)]


@pytest.mark.parametrize("solve", TM_SOLVES,
                         ids=["%s-%x" % s for s in TM_SOLVES])
def test_twisted_solves(w, solve):
    """8^3 x 16, exp(i 0.3 H) links, kappa = 0.15 (past the Wilson operator's
    critical point for these fields) with mu = 0.05: the twist keeps M(mu)
    away from singular. Every solution meets the oracle's twisted residual
    and agrees with the oracle's own CGNR solution within cond(M) tol."""
    solver, flags = solve
    dims, kappa, mu = (8, 8, 8, 16), 0.15, 0.05
    U = synth.gauge_smooth(dims, 0.3, 0)
    b = synth.gaussian_spinor(dims, 1)
    G = w.pack_gauge(U, dims, flags & 0x4)
    B = w.pack_spinor(b, dims)
    X = w.empty_spinor(dims)
    fn = w.solve_cg_tm if solver == "cg" else w.solve_bicgstab_tm
    st = fn(G, B, X, dims, kappa, mu, maxiter=40000, flags=flags)
    assert st["status"] == 0, st
    x = gu.to_np(w.unpack_spinor(X, dims))
    res = oracle.true_residual_tm(U, b, x, dims, kappa, mu)
    assert res <= 1e-10 and abs(res - st["true_res"]) <= 1e-12, (res, st)
    xs, ost = oracle.cgnr_tm(U, b, dims, kappa, mu, tol=1e-12)
    assert ost["status"] == 0
    # sigma_min(M(mu)) >= 2 kappa mu for gamma5-Hermitian D_W: a bound on cond
    cond = (1 + 8 * kappa + 2 * kappa * mu) / (2 * kappa * mu)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    assert err <= cond * (res + 1e-12), (err, cond)
