"""Brute-force dense Wilson-Dirac matrix for tiny lattices (test helper).

An independent way of writing the operator: the 12V x 12V matrix is assembled
block by block from Kronecker products ``spin (4x4) (x) colour (3x3)``, with
``+=`` so that coinciding neighbours on extent-2 directions add. Vector index
``12*s + 3*spin + colour``. Used only to pin the oracle.
"""
import numpy as np

from paper_1112_5280_amd.synth import site_index


def coords(dims):
    lx, ly, lz, lt = dims
    out = []
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    out.append((x, y, z, t))
    return out


def dense_dslash(U, dims, gammas, phases):
    """Dense D_W: sum over bonds of (1 -/+ gamma) (x) U or U^dagger blocks."""
    V = int(np.prod(dims))
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    one = np.eye(4)
    for s, c in enumerate(coords(dims)):
        for mu in range(4):
            cf = list(c)
            cb = list(c)
            cf[mu] = (c[mu] + 1) % dims[mu]
            cb[mu] = (c[mu] - 1) % dims[mu]
            sf = site_index(dims, *cf)
            sb = site_index(dims, *cb)
            pf = phases[mu] if c[mu] == dims[mu] - 1 else 1.0
            pb = np.conj(phases[mu]) if c[mu] == 0 else 1.0
            D[12 * s:12 * s + 12, 12 * sf:12 * sf + 12] += \
                pf * np.kron(one - gammas[mu], U[s, mu])
            D[12 * s:12 * s + 12, 12 * sb:12 * sb + 12] += \
                pb * np.kron(one + gammas[mu], np.conj(U[sb, mu]).T)
    return D


def parity_index(dims):
    """Indices of the even and odd entries of a 12V vector."""
    par = np.array([sum(c) % 2 for c in coords(dims)])
    even_sites = np.nonzero(par == 0)[0]
    odd_sites = np.nonzero(par == 1)[0]
    ev = (12 * even_sites[:, None] + np.arange(12)[None, :]).reshape(-1)
    od = (12 * odd_sites[:, None] + np.arange(12)[None, :]).reshape(-1)
    return ev, od
