"""Meson correlators C_Gamma(t) of Eq. 1 (paper Sec. 4) on the GPU against the
oracle's contraction: on random fields standing in for the 12 propagator
columns (ragged lattices, every Gamma_n), and on the 12 point-source
propagators of an actual batched solve, whose pion channel must equal
-sum |S|^2 per time slice."""
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


def _pack_props(w, cols, dims):
    B = w.empty_batch(dims, 12)
    for r in range(12):
        w.batch_field(B, dims, 0, r).copy_(w.pack_spinor(cols[r], dims))
    return B


@pytest.mark.parametrize("dims,t0", [((4, 4, 4, 4), 0), ((6, 4, 6, 10), 7), ((8, 6, 2, 4), 3)],
                         ids=["4^4", "6x4x6x10", "8x6x2x4"])
def test_contraction_matches_oracle(w, dims, t0):
    cols = np.stack([synth.gaussian_spinor(dims, 300 + r) for r in range(12)])
    B = _pack_props(w, cols, dims)
    got = gu.to_np(w.meson_correlators(B, dims, t0))
    want = oracle.meson(cols, dims, t0)
    assert got.shape == want.shape == (16, dims[3])
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-13, err
    again = gu.to_np(w.meson_correlators(B, dims, t0))
    assert np.array_equal(got, again)


def test_point_source_propagator_correlators(w):
    """8^3 x 16, exp(i 0.3 H) links, kappa = 0.13: the 12 point-source solves
    (batched eo-CG, oracle residual <= 1e-10 each), then their correlators."""
    dims, kappa = (8, 8, 8, 16), 0.13
    U = synth.gauge_smooth(dims, 0.3, 0)
    site = synth.random_site(dims, 2)
    t0 = site // (dims[0] * dims[1] * dims[2])
    srcs = [synth.point_source(dims, site, r // 3, r % 3) for r in range(12)]
    G = w.pack_gauge(U, dims)
    B = _pack_props(w, srcs, dims)
    X = w.empty_batch(dims, 12)
    code, st = w.solve_cg_batch(G, B, X, 12, dims, kappa, flags=w.EO)
    assert code == 0, st
    cols = np.stack([gu.to_np(w.unpack_spinor(w.batch_field(X, dims, 0, r), dims))
                     for r in range(12)])
    for r in (0, 7, 11):
        assert oracle.true_residual(U, srcs[r], cols[r], dims, kappa) <= 1e-10
    got = gu.to_np(w.meson_correlators(X, dims, t0))
    want = oracle.meson(cols, dims, t0)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # pion channel: -sum |S|^2 over each time slice, largest at the source
    V3 = dims[0] * dims[1] * dims[2]
    a2 = (np.abs(cols) ** 2).sum(axis=(0, 2, 3)).reshape(dims[3], V3).sum(axis=1)
    pion = -np.roll(a2, -t0)
    assert np.allclose(got[15].real, pion, rtol=1e-12, atol=0)
    assert np.abs(got[15].imag).max() <= 1e-12 * np.abs(pion).max()
    assert np.argmin(got[15].real) == 0


def test_correlator_argument_errors(w):
    dims = (4, 4, 4, 4)
    B = w.empty_batch(dims, 12)
    with pytest.raises(w.WilsonError):
        w.meson_correlators(B, dims, t0=4)
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(w.WilsonError) as e:
        w.meson_correlators(B, dims, 0, work=small)
    assert e.value.code == w.EWORKSPACE
