"""Uneven batches of independent problems: lattices of several sizes, each with
its own Haar-random gauge field and kappa, solved by one call.

Each solution must equal the solution of the same problem solved alone
bitwise (a problem's kernels, partial sums and reduction order do not depend
on its batch mates), and must meet the FP64 residual bound recomputed by the
CPU oracle with that problem's own gauge field and kappa.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_5280_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

SIZES = ((4, 4, 4, 4), (8, 8, 8, 8), (8, 8, 8, 16))


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


def draw(n, seed, sizes=SIZES):
    """n problems: size uniform over `sizes`, kappa uniform in [0.10, 0.14],
    Haar gauge field and Gaussian source with their own seeds."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        dims = sizes[rng.integers(len(sizes))]
        kappa = float(rng.uniform(0.10, 0.14))
        out.append(dict(dims=dims, kappa=kappa, U=synth.gauge_haar(dims, 1000 + i),
                        b=synth.gaussian_spinor(dims, 5000 + i)))
    return out


def build(w, specs, flags):
    probs = []
    for s in specs:
        G = w.pack_gauge(s["U"], s["dims"], flags & w.LINK12)
        B = w.pack_spinor(s["b"], s["dims"])
        X = w.zeros_spinor(s["dims"])
        probs.append(w.Problem(s["dims"], s["kappa"], G, B, X))
    return probs


def check_against_solo(w, specs, probs, stats, flags, tol=1e-10):
    one = {}
    for i, (s, p) in enumerate(zip(specs, probs)):
        assert stats[i]["status"] == 0, (i, stats[i])
        x = gu.to_np(w.unpack_spinor(p.x, s["dims"]))
        res = oracle.true_residual(s["U"], s["b"], x, s["dims"], s["kappa"])
        assert res <= tol, (i, s["dims"], s["kappa"], res)
        if s["dims"] not in one:
            one[s["dims"]] = w.empty_spinor(s["dims"])
        st = w.solve_cg(p.gauge, p.b, one[s["dims"]], s["dims"], s["kappa"], flags=flags)
        assert st["status"] == 0
        assert st["iterations"] == stats[i]["iterations"], (i, st, stats[i])
        assert np.array_equal(gu.to_np(w.unpack_spinor(one[s["dims"]], s["dims"])), x), i


@pytest.mark.parametrize("flags", [0x20, 0x0, 0x20 | 0x4 | 0x100, 0x20 | 0x40, 0x20 | 0x40 | 0x2],
                         ids=["eo", "full", "eo-link12-graph", "eo-mixed-f32", "eo-mixed-f16"])
def test_mixed_sizes_equal_solo_solves(w, flags):
    specs = draw(12, seed=7)
    probs = build(w, specs, flags)
    code, stats = w.solve_cg_problems(probs, flags=flags)
    assert code == 0, stats
    check_against_solo(w, specs, probs, stats, flags)


def test_uneven_batch_of_64_lattices(w):
    """64 lattices drawn from {4^4, 8^4, 8^3x16}, kappa in [0.10, 0.14]."""
    flags = 0x20
    specs = draw(64, seed=11)
    probs = build(w, specs, flags)
    code, stats = w.solve_cg_problems(probs, flags=flags)
    assert code == 0
    for i, s in enumerate(specs):
        assert stats[i]["status"] == 0
        x = gu.to_np(w.unpack_spinor(probs[i].x, s["dims"]))
        assert oracle.true_residual(s["U"], s["b"], x, s["dims"], s["kappa"]) <= 1e-10, i
    # spot-check a few against their solo solves
    pick = [0, 21, 42, 63]
    check_against_solo(w, [specs[i] for i in pick], [probs[i] for i in pick],
                       [stats[i] for i in pick], flags)


def test_more_than_one_group_per_size_and_initial_guess(w):
    """66 problems of one size split into groups of at most 64; WL_X0 starts
    from the given x (here the exact solution of problem 0, which then needs no
    iteration), and a zero source gives x = 0."""
    dims = (4, 4, 4, 4)
    specs = draw(66, seed=3, sizes=(dims,))
    specs[5]["b"] = np.zeros_like(specs[5]["b"])
    probs = build(w, specs, 0x20)
    code, stats = w.solve_cg_problems(probs, flags=0x20)
    assert code == 0
    assert not gu.to_np(w.unpack_spinor(probs[5].x, dims)).any()
    for i in (0, 63, 64, 65):
        x = gu.to_np(w.unpack_spinor(probs[i].x, dims))
        assert oracle.true_residual(specs[i]["U"], specs[i]["b"], x, dims,
                                    specs[i]["kappa"]) <= 1e-10, i
    x0 = probs[0].x.clone()
    probs2 = build(w, specs[:2], 0x20)
    probs2[0].x.copy_(x0)
    code, stats2 = w.solve_cg_problems(probs2, flags=0x20 | 0x80)
    assert code == 0
    assert stats2[0]["iterations"] == 0
    assert torch.equal(probs2[0].x, x0)
    assert stats2[1]["iterations"] == stats[1]["iterations"]


def test_problem_errors(w):
    specs = draw(2, seed=1)
    probs = build(w, specs, 0)
    probs[1].x = probs[1].b
    with pytest.raises(w.WilsonError):
        w.solve_cg_problems(probs)
    with pytest.raises(w.WilsonError):
        w.solve_cg_problems(build(w, specs, 0), flags=w.F32)


def test_tuned_shared_gauge_shape_never_reaches_per_problem_gauges(w):
    """A shared-gauge batch at 16^3 x 32 (time slices of whole site blocks, so
    its launches are autotuned and may settle on several RHS per thread) runs
    first; then 4 problems of the same size, each with its own gauge field, are
    solved together. Each must use its own links: every solution meets the
    oracle's residual with that problem's field, and equals its solo solve."""
    dims = (16, 16, 16, 32)
    U0 = synth.gauge_haar(dims, 50)
    G0 = w.pack_gauge(U0, dims)
    n = 4
    B = w.empty_batch(dims, n)
    for r in range(n):
        w.batch_field(B, dims, 0, r).copy_(w.pack_spinor(synth.gaussian_spinor(dims, 60 + r), dims))
    X = w.empty_batch(dims, n)
    code, _ = w.solve_cg_batch(G0, B, X, n, dims, 0.12, flags=w.EO)
    assert code == 0
    assert "gauges=shared" in w.tuning_report()
    specs = [dict(dims=dims, kappa=0.11 + 0.005 * i, U=synth.gauge_haar(dims, 70 + i),
                  b=synth.gaussian_spinor(dims, 80 + i)) for i in range(n)]
    probs = build(w, specs, w.EO)
    code, stats = w.solve_cg_problems(probs, flags=w.EO)
    assert code == 0, stats
    check_against_solo(w, specs, probs, stats, w.EO)
