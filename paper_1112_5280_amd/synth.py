"""Seeded synthetic inputs: gauge fields and source spinors.

This module only draws inputs. It holds none of the Wilson-Dirac arithmetic,
so both the CPU oracle (through the tests) and the HIP path can be fed from it.

Canonical layouts (the convention every other part of the repository uses):

* lattice extents ``dims = (Lx, Ly, Lz, Lt)``; site index
  ``x + Lx*(y + Ly*(z + Lz*t))``;
* gauge field: complex128 array ``U[V, 4, 3, 3]``; ``U[s, mu]`` is the SU(3)
  link on the bond from site ``s`` to ``s + mu_hat`` (row-major colour matrix);
* spinor: complex128 array ``psi[V, 4, 3]`` (spin, colour).

Random streams: ``numpy.random.default_rng(seed)`` (PCG64). Every generator
draws all real parts of its complex Gaussian array first, then all imaginary
parts, in C order of the output shape.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "site_index", "site_coords", "gauge_unit", "gauge_haar",
    "gauge_smooth", "haar_su3", "gaussian_spinor", "point_source",
    "random_site", "config_workloads",
]

_CHUNK = 1 << 20  # matrices per batched LAPACK call, bounds peak memory


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def site_index(dims, x, y, z, t):
    lx, ly, lz, _ = dims
    return x + lx * (y + ly * (z + lz * t))


def site_coords(dims, s):
    """Inverse of :func:`site_index`; works on scalars and integer arrays."""
    lx, ly, lz, _ = dims
    x = s % lx
    r = s // lx
    y = r % ly
    r = r // ly
    z = r % lz
    t = r // lz
    return x, y, z, t


def _complex_gauss(rng, shape):
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def haar_su3(n: int, rng) -> np.ndarray:
    """``n`` Haar-distributed SU(3) matrices.

    QR of a complex Gaussian matrix with the phases of R's diagonal moved into
    Q gives a Haar U(3) matrix; dividing by the principal cube root of its
    determinant puts it in SU(3) (the Haar measure is invariant under the
    centre, so any root would do).
    """
    z = _complex_gauss(rng, (n, 3, 3)) / np.sqrt(2.0)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for a in range(0, n, _CHUNK):
        b = min(n, a + _CHUNK)
        q, r = np.linalg.qr(z[a:b])
        d = np.diagonal(r, axis1=1, axis2=2)
        q = q * (d / np.abs(d))[:, None, :]
        det = np.linalg.det(q)
        root = np.exp(1j * np.angle(det) / 3.0)
        out[a:b] = q / root[:, None, None]
    return out


def gauge_unit(dims) -> np.ndarray:
    v = volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1.0
    return u


def gauge_haar(dims, seed: int) -> np.ndarray:
    """Independent Haar SU(3) link on every bond (a maximally rough field)."""
    v = volume(dims)
    rng = np.random.default_rng(seed)
    return haar_su3(v * 4, rng).reshape(v, 4, 3, 3)


def gauge_smooth(dims, eps: float, seed: int) -> np.ndarray:
    """Links ``exp(i*eps*H)`` with ``H`` a random traceless Hermitian matrix.

    ``A`` has independent standard-normal real and imaginary parts,
    ``H = (A + A^dagger)/2 - tr(.)/3``; the exponential is taken through the
    eigendecomposition of ``H``, so each link is unitary with determinant
    ``exp(i*eps*tr H) = 1`` to rounding. At ``eps = 0.3`` the mean plaquette
    is about 0.61, at ``eps = 0.35`` about 0.51.
    """
    v = volume(dims)
    n = v * 4
    rng = np.random.default_rng(seed)
    a = _complex_gauss(rng, (n, 3, 3))
    out = np.empty((n, 3, 3), dtype=np.complex128)
    eye = np.eye(3)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        blk = a[s:e]
        h = 0.5 * (blk + np.conj(np.swapaxes(blk, 1, 2)))
        tr = np.trace(h, axis1=1, axis2=2).real / 3.0
        h = h - tr[:, None, None] * eye
        w, vec = np.linalg.eigh(h)
        ph = np.exp(1j * eps * w)
        out[s:e] = (vec * ph[:, None, :]) @ np.conj(np.swapaxes(vec, 1, 2))
    return out.reshape(v, 4, 3, 3)


def gaussian_spinor(dims, seed: int) -> np.ndarray:
    """Complex Gaussian source: real and imaginary parts ~ N(0, 1)."""
    v = volume(dims)
    rng = np.random.default_rng(seed)
    return _complex_gauss(rng, (v, 4, 3))


def point_source(dims, site: int, spin: int, colour: int) -> np.ndarray:
    """Unit point source at ``site`` in one spin-colour component."""
    psi = np.zeros((volume(dims), 4, 3), dtype=np.complex128)
    psi[site, spin, colour] = 1.0
    return psi


def random_site(dims, seed: int) -> int:
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, volume(dims)))


def config_workloads():
    """The named synthetic workloads (lattice, kappa, gauge generator).

    Seeds: gauge field 0, Gaussian source 1, point-source site 2.
    """
    return {
        "haar4": dict(dims=(4, 4, 4, 4), kappa=0.12, gauge=("haar", None)),
        "smooth16x32": dict(dims=(16, 16, 16, 32), kappa=0.15,
                            gauge=("smooth", 0.3)),
        "smooth32x64": dict(dims=(32, 32, 32, 64), kappa=0.155,
                            gauge=("smooth", 0.35)),
        "smooth24x48": dict(dims=(24, 24, 24, 48), kappa=0.15,
                            gauge=("smooth", 0.3)),
    }
