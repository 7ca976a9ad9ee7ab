"""Solves whose Krylov chunks are captured once into a HIP graph and replayed.

Every replay is followed by the host's read of the solver status (eager work
and a synchronisation between replays); the solution and the iteration count
must equal those of the directly launched solve bitwise, for every solver
variant, and a second graph solve on the same library stream must too.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_5280_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


CASES = [("cg", 0x20), ("cg", 0x0), ("cg", 0x60), ("cg", 0x62), ("bicgstab", 0x20),
         ("bicgstab", 0x60)]


@pytest.mark.parametrize("case", CASES, ids=["cg-eo", "cg-full", "cg-eo-mixed",
                                             "cg-eo-mixed-f16", "bicgstab-eo",
                                             "bicgstab-eo-mixed"])
def test_graph_replay_equals_direct(w, case):
    solver, flags = case
    dims = (4, 4, 4, 8)
    kappa = 0.13
    U = synth.gauge_smooth(dims, 0.3, 3)
    b = synth.gaussian_spinor(dims, 4)
    G = w.pack_gauge(U, dims)
    B = w.pack_spinor(b, dims)
    fn = w.solve_cg if solver == "cg" else w.solve_bicgstab
    X0 = w.zeros_spinor(dims)
    st0 = fn(G, B, X0, dims, kappa, flags=flags)
    ref = gu.to_np(w.unpack_spinor(X0, dims))
    assert st0["status"] == 0
    for _ in range(2):
        X1 = w.zeros_spinor(dims)
        st1 = fn(G, B, X1, dims, kappa, flags=flags | w.GRAPH)
        assert st1["status"] == 0 and st1["iterations"] == st0["iterations"], (st0, st1)
        assert np.array_equal(gu.to_np(w.unpack_spinor(X1, dims)), ref)
    assert oracle.true_residual(U, b, ref, dims, kappa) <= 1e-10


def test_graph_batch_equals_direct(w):
    dims = (4, 4, 4, 8)
    kappa = 0.13
    U = synth.gauge_smooth(dims, 0.3, 5)
    site = synth.random_site(dims, 2)
    srcs = [synth.point_source(dims, site, s, c) for s in range(4) for c in range(3)]
    n = len(srcs)
    G = w.pack_gauge(U, dims)
    B = w.empty_batch(dims, n)
    for r, s in enumerate(srcs):
        w.batch_field(B, dims, 0, r).copy_(w.pack_spinor(s, dims))
    X0, X1 = w.empty_batch(dims, n), w.empty_batch(dims, n)
    c0, s0 = w.solve_cg_batch(G, B, X0, n, dims, kappa, flags=w.EO)
    c1, s1 = w.solve_cg_batch(G, B, X1, n, dims, kappa, flags=w.EO | w.GRAPH)
    assert c0 == 0 and c1 == 0
    for r in range(n):
        a = gu.to_np(w.unpack_spinor(w.batch_field(X0, dims, 0, r), dims))
        c = gu.to_np(w.unpack_spinor(w.batch_field(X1, dims, 0, r), dims))
        assert np.array_equal(a, c) and s0[r]["iterations"] == s1[r]["iterations"]
