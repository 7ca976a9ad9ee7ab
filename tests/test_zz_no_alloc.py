"""solve_cg_noalloc: the solve with the library's static scratch instead of a
caller workspace gives the bits of solve_cg with a workspace, on two calls in
a row (the second on a smaller lattice, so stale scratch contents of the
first must not matter), and allocates no device memory once warm."""
import ctypes

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


def _noalloc(w, G, B, X, dims, kappa, flags):
    """solve_cg_noalloc called through the C ABI directly."""
    st = w.SolveStats()
    code = w.lib.solve_cg_noalloc(w._ptr(G), w._ptr(B), w._ptr(X), w._dims(dims), float(kappa),
                                  w._phases(w.ANTIPERIODIC_T), 1e-10, 20000, flags,
                                  ctypes.byref(st), w._stream(None))
    return code, st.as_dict()


CASES = [((8, 8, 8, 16), 0.15, 0x20), ((4, 4, 4, 4), 0.12, 0x20 | 0x40),
         ((8, 8, 8, 8), 0.14, 0x20 | 0x40 | 0x2), ((4, 4, 4, 4), 0.12, 0x0)]


def test_noalloc_equals_workspace_solve(w):
    for dims, kappa, flags in CASES:     # larger lattice first, then smaller
        U = synth.gauge_smooth(dims, 0.3, 3) if dims[0] == 8 else synth.gauge_haar(dims, 0)
        b = synth.gaussian_spinor(dims, 4)
        G = w.pack_gauge(U, dims)
        B = w.pack_spinor(b, dims)
        X1, X2 = w.empty_spinor(dims), w.empty_spinor(dims)
        ref = w.solve_cg(G, B, X1, dims, kappa, maxiter=20000, flags=flags)
        code, st = _noalloc(w, G, B, X2, dims, kappa, flags)
        assert code == 0 and ref["status"] == 0, (dims, flags, code, st, ref)
        assert st["iterations"] == ref["iterations"], (dims, flags, st, ref)
        assert torch.equal(X1, X2), (dims, flags)
        x = gu.to_np(w.unpack_spinor(X2, dims))
        res = oracle.true_residual(U, b, x, dims, kappa)
        assert res <= 1e-10 and abs(res - st["true_res"]) <= 1e-12, (dims, flags, res, st)


def test_noalloc_allocates_no_device_memory_once_warm(w):
    dims, kappa = (8, 8, 8, 8), 0.13
    U = synth.gauge_smooth(dims, 0.3, 5)
    G = w.pack_gauge(U, dims)
    B = w.pack_spinor(synth.gaussian_spinor(dims, 6), dims)
    X = w.empty_spinor(dims)
    for flags in (0x20, 0x20 | 0x40):
        assert _noalloc(w, G, B, X, dims, kappa, flags)[0] == 0   # warm-up
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for flags in (0x20, 0x20 | 0x40, 0x20, 0x20 | 0x40):
        assert _noalloc(w, G, B, X, dims, kappa, flags)[0] == 0
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
