"""Helpers shared by the GPU parity tests (test infrastructure)."""
import numpy as np

import oracle
import torch

# Bars from the problem statement: FP64 operators agree with the FP64 oracle to
# 1e-13 relative; FP32 to 1e-6. Both the field-norm ratio and the max-abs ratio
# must meet them (sites can be near zero, so no per-site relative error).
# FP16 storage has no stated bar; binary16's unit roundoff is 2^-11 = 4.9e-4,
# the inputs are rounded once (spinors relative to their site maximum, links
# absolutely), the 12-real rebuild multiplies two rounded entries, and the
# output is rounded once more, so the error is a few units of 4.9e-4: the bar
# 3e-3 allows six.
TOL = {0x0: 1e-13, 0x1: 1e-6, 0x2: 3e-3}


def errs(got, want):
    got = np.asarray(got).reshape(-1)
    want = np.asarray(want).reshape(-1)
    d = got - want
    return (float(np.linalg.norm(d) / np.linalg.norm(want)),
            float(np.abs(d).max() / np.abs(want).max()))


def assert_close(got, want, tol, what=""):
    n, m = errs(got, want)
    assert n <= tol and m <= tol, "%s: rel-norm %.3e, rel-max %.3e > %.1e" % (what, n, m, tol)


def sync():
    torch.cuda.synchronize()


def to_np(t):
    return t.detach().cpu().numpy()


def half_to_canon(w, half, dims, flags, parity):
    """Unpack one packed parity block into a canonical [V,4,3] array (zeros on
    the other parity)."""
    prec = flags & 0x3
    full = w.zeros_spinor(dims, prec, 2)
    w.parity_block(full, dims, prec, parity).copy_(half)
    return to_np(w.unpack_spinor(full, dims, prec))


def parity_of_sites(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return ((x + y + z + t) % 2).reshape(-1)


def heatbath_spread(U0, dims, beta, nsweeps, sweep0, seed):
    """How far the oracle's own chain moves when every element of its start is
    perturbed by one part in 1e16 (about one ulp). The heat bath amplifies
    rounding: a link's new value depends on the direction b/|b| of its staple
    term, ill conditioned where |b| is small (strong coupling, rough fields),
    and each update feeds the staples of the next. Measured on the CPU: after
    3 sweeps about 6e-14 at beta 5.7, 6e-10 at beta 2, 9e-7 at beta 0.5."""
    rng = np.random.default_rng(2024)
    a = U0.copy()
    oracle.heatbath(a, dims, beta, nsweeps, sweep0=sweep0, seed=seed)
    b = U0 * (1 + 1e-16 * rng.standard_normal(U0.shape))
    oracle.heatbath(b, dims, beta, nsweeps, sweep0=sweep0, seed=seed)
    return a, float(np.abs(a - b).max())
