"""Solvers on canonical fields (WL_CANON): the library packs the complex128
gauge field and spinors into its workspace, solves, and unpacks x. The result
is bitwise the solve on fields packed by the caller, for every solver mode,
with and without an initial guess; the batched and allocation-free entry
points refuse the flag."""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_5280_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

DIMS, KAPPA = (6, 4, 6, 10), 0.13


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


@pytest.fixture(scope="module")
def fields():
    return synth.gauge_smooth(DIMS, 0.3, 4), synth.gaussian_spinor(DIMS, 5)


MODES = [("cg", 0x20), ("cg", 0x20 | 0x40), ("cg", 0x20 | 0x40 | 0x2), ("cg", 0x20 | 0x4),
         ("cg", 0x0), ("bicgstab", 0x20), ("bicgstab", 0x20 | 0x40), ("cg_tm", 0x20 | 0x40)]


@pytest.mark.parametrize("solver,flags", MODES,
                         ids=["%s-%#x" % (s, f) for s, f in MODES])
def test_canonical_equals_packed(w, fields, solver, flags):
    U, b = fields
    Ud = torch.from_numpy(U).to("cuda")
    bd = torch.from_numpy(b).to("cuda")
    G = w.pack_gauge(U, DIMS, flags & 0x4)
    B = w.pack_spinor(b, DIMS)

    def run(g, bb, xx, f):
        if solver == "cg_tm":
            return w.solve_cg_tm(g, bb, xx, DIMS, KAPPA, 0.05, tol=1e-10, maxiter=5000, flags=f)
        fn = w.solve_cg if solver == "cg" else w.solve_bicgstab
        return fn(g, bb, xx, DIMS, KAPPA, tol=1e-10, maxiter=5000, flags=f)

    X = w.empty_spinor(DIMS)
    st_p = run(G, B, X, flags)
    want = w.unpack_spinor(X, DIMS)
    xd = torch.empty_like(bd)
    st_c = run(Ud, bd, xd, flags | w.CANON)
    assert st_p["status"] == 0 and st_c["status"] == 0, (st_p, st_c)
    assert torch.equal(xd, want)
    assert st_c["iterations"] == st_p["iterations"]
    assert st_c["true_res"] == st_p["true_res"]
    if solver != "cg_tm":
        assert oracle.true_residual(U, b, gu.to_np(xd), DIMS, KAPPA) <= 1e-10
    # an initial guess in canonical layout (the solution itself: no iterations)
    st_0 = run(Ud, bd, xd, flags | w.CANON | w.X0)
    assert st_0["status"] == 0 and st_0["iterations"] == 0
    assert torch.equal(xd, want)


def test_canonical_refused_where_it_does_not_apply(w, fields):
    U, b = fields
    Ud = torch.from_numpy(U).to("cuda")
    bd = torch.from_numpy(b).to("cuda")
    xd = torch.empty_like(bd)
    assert w.workspace_bytes(DIMS, w.EO | w.CANON, 2) == 0
    with pytest.raises(w.WilsonError):
        w.solve_cg_noalloc(Ud, bd, xd, DIMS, KAPPA, flags=w.EO | w.CANON)
    B = w.empty_batch(DIMS, 2)
    X = w.empty_batch(DIMS, 2)
    G = w.pack_gauge(U, DIMS)
    with pytest.raises(w.WilsonError):
        w.solve_cg_batch(G, B, X, 2, DIMS, KAPPA, flags=w.EO | w.CANON,
                         work=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
