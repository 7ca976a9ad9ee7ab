"""Calls on a side stream are ordered after the work already queued on the
current stream: an input written there by a slow producer is read complete,
and buffers the binding allocates for the call stay reserved for the side
stream."""
import numpy as np
import pytest
import torch

from paper_1112_5280_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 8, 16)


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


def _busy_current_stream():
    # some milliseconds of FP32 products queued on the current stream
    a = torch.full((2048, 2048), 1e-3, dtype=torch.float32, device="cuda")
    for _ in range(30):
        a = a @ a
    return a


def test_side_stream_sees_current_stream_writes(w):
    psi = synth.gaussian_spinor(DIMS, 3)
    P = w.pack_spinor(psi, DIMS)
    Q = torch.zeros_like(P)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    _busy_current_stream()
    Q.copy_(P)                                   # the producer, behind the products
    out = w.unpack_spinor(Q, DIMS, stream=side)  # output allocated here, used on `side`
    side.synchronize()
    # pack and unpack move FP64 values unchanged
    assert np.array_equal(out.cpu().numpy(), psi)
    torch.cuda.synchronize()


def test_side_stream_solve_and_correlators(w):
    """A solve and a contraction on a side stream, each with buffers the binding
    allocates, give the results of the same calls on the current stream."""
    U = synth.gauge_smooth(DIMS, 0.3, 1)
    b = synth.gaussian_spinor(DIMS, 2)
    G = w.pack_gauge(U, DIMS)
    B = w.pack_spinor(b, DIMS)
    X0 = w.empty_spinor(DIMS)
    st0 = w.solve_cg(G, B, X0, DIMS, 0.12, flags=w.EO)
    side = torch.cuda.Stream()
    X1 = w.empty_spinor(DIMS)
    torch.cuda.synchronize()
    _busy_current_stream()
    X1.fill_(7)                                  # overwritten by the solve, after this fill
    st1 = w.solve_cg(G, B, X1, DIMS, 0.12, flags=w.EO, stream=side)
    side.synchronize()
    assert st0["status"] == st1["status"] == 0
    assert torch.equal(X0, X1)

    props = w.empty_batch(DIMS, 12)
    for r in range(12):
        w.batch_field(props, DIMS, 0, r).copy_(B)
    c0 = w.meson_correlators(props, DIMS, 0).cpu()
    torch.cuda.synchronize()
    _busy_current_stream()
    c1 = w.meson_correlators(props, DIMS, 0, stream=side)
    side.synchronize()
    assert torch.equal(c0, c1.cpu())
    torch.cuda.synchronize()
