"""Launch shapes of the hop kernel (RHS per thread, chunked RHS-group order,
tile groups walked through time) reorder work but change no arithmetic:
every shape gives bitwise the same operator outputs and the same solves,
reductions included, and the autotuned shapes give the same bits again."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1112_5280_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

# Lx/2 * Ly * Lz = 1024 column sites per slice: 4 blocks per time slice
DIMS = (16, 16, 8, 8)
SHAPES = ["1,1,0", "1,1,1", "1,1,2", "2,1,1", "3,4,2", "4,64,0", "2,1000000,1"]


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


@pytest.fixture(scope="module")
def inputs(w):
    U = synth.gauge_smooth(DIMS, 0.3, 11)
    srcs = [synth.gaussian_spinor(DIMS, 60 + r) for r in range(5)]
    return U, srcs


def run_all(w, U, srcs):
    """Operator outputs (full M, M^dag batch, eo hop) and an eo CG solve."""
    kappa = 0.13
    out = []
    for flags in (0x0, 0x1):
        prec = flags & 0x3
        G = w.pack_gauge(U, DIMS, flags)
        P = w.pack_spinor(srcs[0], DIMS, prec)
        O = w.empty_spinor(DIMS, prec)
        w.wilson_dslash(G, P, O, DIMS, kappa, flags=flags)
        out.append(w.unpack_spinor(O, DIMS, prec))
        n = len(srcs)
        B = w.empty_batch(DIMS, n, prec)
        for r, s in enumerate(srcs):
            w.batch_field(B, DIMS, prec, r).copy_(w.pack_spinor(s, DIMS, prec))
        OB = w.empty_batch(DIMS, n, prec)
        w.wilson_dslash_batch(G, B, OB, n, DIMS, kappa, flags=flags | 0x8)
        out += [w.unpack_spinor(w.batch_field(OB, DIMS, prec, r), DIMS, prec) for r in range(n)]
        Oh = w.empty_spinor(DIMS, prec, 1)
        w.wilson_dslash_eo(G, w.parity_block(P, DIMS, prec, 1), Oh, DIMS, kappa, 0,
                           flags=flags | 0x10)
        out.append(Oh.clone())
    G = w.pack_gauge(U, DIMS)
    B = w.pack_spinor(srcs[1], DIMS)
    for flags in (0x20, 0x20 | 0x40):
        X = w.empty_spinor(DIMS)
        st = w.solve_cg(G, B, X, DIMS, kappa, flags=flags)
        assert st["status"] == 0
        out.append(w.unpack_spinor(X, DIMS))
    n = 4
    BB = w.empty_batch(DIMS, n)
    for r in range(n):
        w.batch_field(BB, DIMS, 0, r).copy_(w.pack_spinor(srcs[r], DIMS))
    XB = w.empty_batch(DIMS, n)
    code, _ = w.solve_cg_batch(G, BB, XB, n, DIMS, kappa, flags=0x20)
    assert code == 0
    out += [w.unpack_spinor(w.batch_field(XB, DIMS, 0, r), DIMS) for r in range(n)]
    gu.sync()
    return [gu.to_np(t) for t in out]


def test_every_shape_gives_the_same_bits(w, inputs):
    U, srcs = inputs
    ref = None
    try:
        for shape in SHAPES:
            os.environ["WL_TUNE_FORCE"] = shape
            got = run_all(w, U, srcs)
            if ref is None:
                ref = got
                continue
            for k, (a, b) in enumerate(zip(ref, got)):
                assert np.array_equal(a, b), (shape, k)
    finally:
        os.environ.pop("WL_TUNE_FORCE", None)
    # the tuned shapes (the tuner times candidates on these very calls)
    got = run_all(w, U, srcs)
    for k, (a, b) in enumerate(zip(ref, got)):
        assert np.array_equal(a, b), ("tuned", k)
    assert "L=16x16x8x8" in w.tuning_report()
    # and the bits are the right operator
    kappa = 0.13
    gu.assert_close(ref[0], oracle.mop(U, srcs[0], DIMS, kappa), gu.TOL[0], "M")
    x = ref[-6]
    assert oracle.true_residual(U, srcs[1], x, DIMS, kappa) <= 1e-10
