"""The CPU oracle against what the mathematics and the physics fix.

Every oracle function is pinned here by something other than itself: closed
forms (free-field plane waves and spectrum), invariants (gamma5 hermiticity,
gauge covariance, even-odd split), a dense operator assembled another way,
LAPACK, and a Neumann series.
"""
import numpy as np
import pytest

import oracle
from paper_1112_5280_amd import synth
from tests import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_generators_are_su3():
    for U in (synth.gauge_haar((2, 2, 2, 4), 0),
              synth.gauge_smooth((2, 2, 2, 4), 0.35, 0)):
        m = U.reshape(-1, 3, 3)
        eye = np.eye(3)
        assert np.abs(m @ np.conj(np.swapaxes(m, 1, 2)) - eye).max() < 1e-14
        assert np.abs(np.linalg.det(m) - 1).max() < 1e-14


def test_smooth_field_plaquette(orc):
    """H drawn as a GUE-normalised traceless Hermitian matrix gives a mean
    plaquette near 0.6 at eps = 0.3 (and near 0.5 at eps = 0.35)."""
    d = (8, 8, 8, 8)
    assert abs(orc.plaquette(synth.gauge_smooth(d, 0.3, 0), d) - 0.611) < 0.01
    assert abs(orc.plaquette(synth.gauge_smooth(d, 0.35, 0), d) - 0.509) < 0.01
    # independent Haar links: <Re tr U_P / 3> = 0
    assert abs(orc.plaquette(synth.gauge_haar(d, 0), d)) < 0.01


def test_generator_determinism():
    a = synth.gauge_smooth((2, 2, 2, 2), 0.3, 4)
    b = synth.gauge_smooth((2, 2, 2, 2), 0.3, 4)
    assert np.array_equal(a, b)
    assert np.array_equal(synth.gaussian_spinor((2, 2, 2, 2), 1),
                          synth.gaussian_spinor((2, 2, 2, 2), 1))
