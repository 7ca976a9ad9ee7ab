"""The configuration chain with measurements (paper Sec. 4: one task generates
configurations by heat bath while the other measures meson correlators on the
previous one). Overlapping the two tasks on two streams must not change any
result: the chain equals the heat bath run in one piece, and every
configuration's correlators equal those of a separate solve on it."""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_5280_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 8)
KAPPA = 0.12
BETA = 5.7


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


@pytest.fixture(scope="module")
def chains(w):
    from paper_1112_5280_amd.ensemble import Ensemble
    U0 = synth.gauge_unit(DIMS)
    out = {}
    for ov in (True, False):
        e = Ensemble(U0, DIMS, BETA, sweeps=2, kappa=KAPPA, site=5, seed=9, overlap=ov)
        corr = e.run(3)
        out[ov] = (corr, gu.to_np(e.U[3 % 2]), e.stats)
    return U0, out


def test_overlap_changes_nothing(chains):
    _, out = chains
    assert torch.equal(out[True][0], out[False][0])
    assert np.array_equal(out[True][1], out[False][1])


def test_chain_is_the_heatbath_in_one_piece(w, chains):
    U0, out = chains
    # after 3 steps of 2 sweeps the newest configuration is U_3 = 6 sweeps of U_0
    Ud = torch.from_numpy(U0.copy()).to("cuda")
    w.heatbath(Ud, DIMS, BETA, nsweeps=6, sweep0=0, seed=9)
    assert np.array_equal(gu.to_np(Ud), out[True][1])
    want = U0.copy()
    oracle.heatbath(want, DIMS, BETA, 6, sweep0=0, seed=9)
    assert np.abs(out[True][1] - want).max() <= 1e-12


def test_correlators_of_each_configuration(w, chains):
    """Configuration k (2k sweeps from the cold start) measured on its own:
    the point-source propagator by the batched solver, then Eq. 1's
    correlators, compared with the chain's; the pion channel (Gamma = g5,
    index 15) is negative and real, as Eq. 1 makes it -sum |S|^2."""
    U0, out = chains
    corr = out[True][0]
    V = int(np.prod(DIMS))
    for k in range(3):
        Uk = U0.copy()
        if k:
            oracle.heatbath(Uk, DIMS, BETA, 2 * k, sweep0=0, seed=9)
        G = w.pack_gauge(Uk, DIMS)
        B = w.empty_batch(DIMS, 12)
        for r in range(12):
            src = np.zeros((V, 4, 3), np.complex128)
            src[5, r // 3, r % 3] = 1.0
            w.pack_spinor(src, DIMS, out=w.batch_field(B, DIMS, 0, r))
        X = w.empty_batch(DIMS, 12)
        code, st = w.solve_cg_batch(G, B, X, 12, DIMS, KAPPA, tol=1e-10, flags=w.EO)
        assert code == w.OK
        c = w.meson_correlators(X, DIMS, 0).cpu()
        # the field here comes from the oracle's heat bath, the chain's from the
        # kernels: equal to rounding, so the correlators agree to solver accuracy
        assert torch.allclose(c, corr[k], rtol=1e-8, atol=1e-12), k
        assert (corr[k][15].real < 0).all() and corr[k][15].imag.abs().max() < 1e-12, k
    assert all(s["status"] == 0 for per_rhs in out[True][2] for s in per_rhs)
