"""GPU parity of the Wilson operator kernels against the FP64 CPU oracle.

Element-by-element comparison on the same seeded inputs for the full-lattice
operator (M, M^dag, D_W, D_W^dag), the even-odd hop D_{p,1-p} and the Schur
complement Mhat_p (and adjoint), in FP64 and FP32, with 18- and 12-real links,
on lattices that span several thread blocks with a ragged tail and on the
degenerate extent-2 lattice; the physics pins run directly on the GPU
operator; the full 32^3 x 64 lattice is checked on sampled sites.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_5280_amd import synth
from tests import gpu_util as gu
from tests.pins import gauge_transform, _momenta, _plane_wave

pytestmark = pytest.mark.gpu

# 2^4: neighbours coincide; 6x4x6x10: 720 sites per parity = 2 blocks + a
# ragged 208-site tail; 8x4x6x12 another ragged shape.
DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 6, 10), (8, 4, 6, 12)]
PHASES = [(1, 1, 1, -1), (np.exp(0.3j), np.exp(-1.2j), 1j, -1)]


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import wilson
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wilson


def _fields(dims, seed):
    return synth.gauge_haar(dims, seed), synth.gaussian_spinor(dims, seed + 100)


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("prec", [0x0, 0x1, 0x2], ids=["f64", "f32", "f16s"])
@pytest.mark.parametrize("link", [0x0, 0x4], ids=["link18", "link12"])
@pytest.mark.parametrize("phases", PHASES, ids=["antiperiodic", "twisted"])
def test_full_operator(w, dims, prec, link, phases):
    kappa = 0.137
    U, psi = _fields(dims, 1)
    G = w.pack_gauge(U, dims, prec | link)
    P = w.pack_spinor(psi, dims, prec)
    out = w.empty_spinor(dims, prec)
    for mode, name in ((0, "M"), (w.DAG, "Mdag"), (w.HOP, "D"), (w.HOP | w.DAG, "Ddag")):
        w.wilson_dslash(G, P, out, dims, kappa, phases, prec | link | mode)
        got = gu.to_np(w.unpack_spinor(out, dims, prec))
        dag = bool(mode & w.DAG)
        if mode & w.HOP:
            want = oracle.dslash(U, psi, dims, phases, dagger=dag)
        else:
            want = oracle.mop(U, psi, dims, kappa, phases, dagger=dag)
        gu.assert_close(got, want, gu.TOL[prec], "%s %s" % (name, dims))


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("prec", [0x0, 0x1, 0x2], ids=["f64", "f32", "f16s"])
@pytest.mark.parametrize("link", [0x0, 0x4], ids=["link18", "link12"])
def test_even_odd(w, dims, prec, link):
    kappa = 0.141
    phases = PHASES[1]
    U, psi = _fields(dims, 2)
    par = gu.parity_of_sites(dims)
    G = w.pack_gauge(U, dims, prec | link)
    P = w.pack_spinor(psi, dims, prec)
    half = w.empty_spinor(dims, prec, 1)
    for p in (0, 1):
        sel = par == p
        for dag in (False, True):
            f = prec | link | (w.DAG if dag else 0)
            # hop D_{p,1-p}: input is the other parity's block
            w.wilson_dslash_eo(G, w.parity_block(P, dims, prec, 1 - p), half, dims, kappa, p,
                               phases, f | w.HOP)
            got = gu.half_to_canon(w, half, dims, prec, p)
            want = oracle.dslash_eo(U, psi, dims, p, phases, dagger=dag)
            gu.assert_close(got[sel], want[sel], gu.TOL[prec], "hop p=%d dag=%d" % (p, dag))
            # Schur complement on parity p: out is a full field whose other
            # parity block receives the intermediate D_{1-p,p} in
            full = w.empty_spinor(dims, prec, 2)
            w.wilson_dslash_eo(G, w.parity_block(P, dims, prec, p), full, dims, kappa, p,
                               phases, f)
            got = gu.half_to_canon(w, w.parity_block(full, dims, prec, p), dims, prec, p)
            psi_p = psi * sel[:, None, None]
            want = oracle.schur(U, psi_p, dims, kappa, p, phases, dagger=dag)
            gu.assert_close(got[sel], want[sel], gu.TOL[prec], "schur p=%d dag=%d" % (p, dag))
            mid = gu.half_to_canon(w, w.parity_block(full, dims, prec, 1 - p), dims, prec, 1 - p)
            want = oracle.dslash_eo(U, psi_p, dims, 1 - p, phases, dagger=dag)
            gu.assert_close(mid[~sel], want[~sel], gu.TOL[prec], "schur intermediate p=%d" % p)


@pytest.mark.parametrize("dims", [(128, 2, 2, 4), (132, 2, 2, 4), (2, 34, 2, 4), (10, 6, 4, 6)],
                         ids=["Lx128-widest-window", "Lx132-no-window", "Lx2-Ly34", "10x6x4x6"])
@pytest.mark.parametrize("prec", [0x0, 0x1], ids=["f64", "f32"])
def test_lds_window_edges(w, dims, prec):
    """The x/y neighbour window of the FP64 and FP32 kernels at its edges: the
    widest row it stages (Lx/2 = 64), a row too wide for it (global loads
    throughout), rows of one site with many y wraps, and blocks that straddle
    rows and end in the padding of the last block; full operator and both
    even-odd hops against the oracle."""
    kappa = 0.133
    phases = PHASES[1]
    U, psi = _fields(dims, 5)
    G = w.pack_gauge(U, dims, prec)
    P = w.pack_spinor(psi, dims, prec)
    out = w.empty_spinor(dims, prec)
    for dag in (False, True):
        w.wilson_dslash(G, P, out, dims, kappa, phases, prec | (w.DAG if dag else 0))
        got = gu.to_np(w.unpack_spinor(out, dims, prec))
        gu.assert_close(got, oracle.mop(U, psi, dims, kappa, phases, dagger=dag), gu.TOL[prec],
                        "M dag=%d %s" % (dag, dims))
    par = gu.parity_of_sites(dims)
    half = w.empty_spinor(dims, prec, 1)
    for p in (0, 1):
        w.wilson_dslash_eo(G, w.parity_block(P, dims, prec, 1 - p), half, dims, kappa, p,
                           phases, prec | w.HOP)
        got = gu.half_to_canon(w, half, dims, prec, p)
        want = oracle.dslash_eo(U, psi, dims, p, phases)
        gu.assert_close(got[par == p], want[par == p], gu.TOL[prec], "hop p=%d %s" % (p, dims))


def test_pack_roundtrip(w):
    dims = (6, 4, 6, 10)
    psi = synth.gaussian_spinor(dims, 7)
    got = gu.to_np(w.unpack_spinor(w.pack_spinor(psi, dims), dims))
    assert np.array_equal(got, psi)
    got32 = gu.to_np(w.unpack_spinor(w.pack_spinor(psi, dims, w.F32), dims, w.F32))
    assert np.array_equal(got32, psi.astype(np.complex64).astype(np.complex128))
    # FP16 storage: each component within half a binary16 ulp of the site maximum
    got16 = gu.to_np(w.unpack_spinor(w.pack_spinor(psi, dims, w.F16S), dims, w.F16S))
    smax = np.maximum(np.abs(psi.real), np.abs(psi.imag)).reshape(len(psi), -1).max(1)
    err = np.maximum(np.abs((got16 - psi).real), np.abs((got16 - psi).imag))
    assert (err.reshape(len(psi), -1).max(1) <= smax * 2.0 ** -11 * (1 + 1e-6)).all()


def test_gauge_pack_roundtrip(w):
    """unpack_gauge inverts pack_gauge: FP64 18-real exactly; FP32 to the
    rounding of the stored values; the 12-real formats give the third row
    rebuilt from the first two, the same unitary link to rounding (the
    generated links have det = 1 to ~1e-15), FP16 to a few binary16 ulps."""
    dims = (6, 4, 6, 10)
    U = synth.gauge_haar(dims, 8)
    assert np.array_equal(gu.to_np(w.unpack_gauge(w.pack_gauge(U, dims), dims)), U)
    got = gu.to_np(w.unpack_gauge(w.pack_gauge(U, dims, w.F32), dims, w.F32))
    assert np.array_equal(got, U.astype(np.complex64).astype(np.complex128))
    for flags, tol in ((w.F64 | w.LINK12, 1e-14), (w.F32 | w.LINK12, 3e-7), (w.F16S, 5e-4),
                       (w.F16S | w.LINK12, 2e-3)):
        got = gu.to_np(w.unpack_gauge(w.pack_gauge(U, dims, flags), dims, flags))
        assert np.abs(got - U).max() <= tol, (flags, np.abs(got - U).max())


def test_f16_storage_far_below_fp32_normal_range(w):
    """Site magnitudes spread over 10^0 .. 10^-44 (into the FP32 denormals, as
    the far sites of a point-source residual are after a few CG iterations),
    plus zero sites: FP16 storage and the FP16 operator stay finite, normal-range
    sites keep the half-ulp bound, and M agrees with the oracle."""
    dims = (6, 4, 6, 10)
    V = synth.volume(dims)
    rng = np.random.default_rng(11)
    psi = synth.gaussian_spinor(dims, 12) * 10.0 ** -rng.uniform(0, 44, V)[:, None, None]
    psi[rng.random(V) < 0.1] = 0
    got = gu.to_np(w.unpack_spinor(w.pack_spinor(psi, dims, w.F16S), dims, w.F16S))
    assert np.isfinite(got).all()
    smax = np.maximum(np.abs(psi.real), np.abs(psi.imag)).reshape(V, -1).max(1)
    err = np.maximum(np.abs((got - psi).real), np.abs((got - psi).imag)).reshape(V, -1).max(1)
    normal = smax >= 2.0 ** -100          # values and scales well inside the FP32 range
    assert (err[normal] <= smax[normal] * 2.0 ** -11 * (1 + 1e-6)).all()
    # below: denormal products may also be flushed to zero
    assert (err[~normal] <= smax[~normal] * 2.0 ** -11 * (1 + 1e-6) + 2.0 ** -126).all()
    assert not got[smax == 0].any()
    U = synth.gauge_haar(dims, 13)
    G = w.pack_gauge(U, dims, w.F16S)
    out = w.empty_spinor(dims, w.F16S)
    w.wilson_dslash(G, w.pack_spinor(psi, dims, w.F16S), out, dims, 0.15, flags=w.F16S)
    got = gu.to_np(w.unpack_spinor(out, dims, w.F16S))
    assert np.isfinite(got).all()
    gu.assert_close(got, oracle.mop(U, psi, dims, 0.15), gu.TOL[0x2], "M on FP16 storage")


def test_free_field_plane_wave_on_gpu(w):
    """Unit links: the GPU operator maps e^{ipx} w to e^{ipx} A(p) w."""
    dims = (4, 6, 2, 8)
    kappa = 0.13
    phases = (np.exp(0.3j), np.exp(-1.1j), 1.0, -1.0)
    g = [oracle.gamma(mu) for mu in range(4)]
    mom = _momenta(dims, phases)
    G = w.pack_gauge(synth.gauge_unit(dims), dims)
    out = w.empty_spinor(dims)
    rng = np.random.default_rng(3)
    for n in [(1, 2, 0, 3), (0, 0, 1, 0), (3, 5, 1, 7)]:
        p = [mom[mu][n[mu]] for mu in range(4)]
        A = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) + \
            2j * kappa * sum(np.sin(p[mu]) * g[mu] for mu in range(4))
        wave = _plane_wave(dims, p)
        wv = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = wave[:, None, None] * wv[None]
        w.wilson_dslash(G, w.pack_spinor(psi, dims), out, dims, kappa, phases)
        got = gu.to_np(w.unpack_spinor(out, dims))
        gu.assert_close(got, wave[:, None, None] * (A @ wv)[None], 1e-13, "plane wave")


def test_gamma5_hermiticity_and_covariance_on_gpu(w):
    dims = (4, 4, 6, 4)
    kappa = 0.12
    U = synth.gauge_haar(dims, 31)
    phi = synth.gaussian_spinor(dims, 32)
    psi = synth.gaussian_spinor(dims, 33)
    G = w.pack_gauge(U, dims)
    out = w.empty_spinor(dims)

    def apply(G_, v, flags=0):
        w.wilson_dslash(G_, w.pack_spinor(v, dims), out, dims, kappa, flags=flags)
        return gu.to_np(w.unpack_spinor(out, dims))

    lhs = np.vdot(phi, apply(G, psi))
    rhs = np.vdot(apply(G, phi, w.DAG), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    omega = synth.haar_su3(synth.volume(dims), np.random.default_rng(34))
    Gg = w.pack_gauge(gauge_transform(U, dims, omega), dims)
    a = apply(Gg, np.einsum("sab,sib->sia", omega, psi))
    b = np.einsum("sab,sib->sia", omega, apply(G, psi))
    gu.assert_close(a, b, 1e-13, "gauge covariance")


def test_deterministic(w):
    dims = (8, 4, 6, 12)
    U, psi = _fields(dims, 5)
    G = w.pack_gauge(U, dims)
    P = w.pack_spinor(psi, dims)
    o1, o2 = w.empty_spinor(dims), w.empty_spinor(dims)
    w.wilson_dslash(G, P, o1, dims, 0.13)
    w.wilson_dslash(G, P, o2, dims, 0.13)
    gu.sync()
    assert torch.equal(o1, o2)


def test_invalid_arguments_enqueue_nothing(w):
    dims = (4, 4, 4, 4)
    G = w.pack_gauge(synth.gauge_unit(dims), dims)
    P = w.pack_spinor(synth.gaussian_spinor(dims, 1), dims)
    with pytest.raises(w.WilsonError):
        w.wilson_dslash(G, P, P, dims, 0.1)                     # aliasing
    with pytest.raises(w.WilsonError):
        w.wilson_dslash(G, P, w.empty_spinor(dims), (4, 4, 4, 5), 0.1)   # odd extent
    with pytest.raises(w.WilsonError):
        w.wilson_dslash_eo(G, P, w.empty_spinor(dims), dims, 0.1, 2)     # bad parity
    with pytest.raises(w.WilsonError):   # Schur mode: in inside out's scratch block
        w.wilson_dslash_eo(G, w.parity_block(P, dims, 0, 1), P, dims, 0.1, 0)


@pytest.fixture(scope="module")
def big_fields():
    dims = (32, 32, 32, 64)
    print("generating the 32^3 x 64 exp(i eps H) field", flush=True)
    return dims, synth.gauge_smooth(dims, 0.35, 0), synth.gaussian_spinor(dims, 1)


@pytest.mark.parametrize("flags", [0x0, 0x1 | 0x4], ids=["f64_link18", "f32_link12"])
def test_full_size_sampled(w, big_fields, flags):
    """32^3 x 64 (the largest configuration): sampled sites against the oracle,
    with the launch configuration the benchmark times."""
    dims, U, psi = big_fields
    kappa = 0.155
    prec = flags & 0x3
    G = w.pack_gauge(U, dims, flags)
    P = w.pack_spinor(psi, dims, prec)
    out = w.empty_spinor(dims, prec)
    w.wilson_dslash(G, P, out, dims, kappa, flags=flags)
    got = gu.to_np(w.unpack_spinor(out, dims, prec))
    V = synth.volume(dims)
    rng = np.random.default_rng(9)
    # random sites plus every corner of the lattice (wrapping hops in all directions)
    corners = [synth.site_index(dims, x, y, z, t) for x in (0, 31) for y in (0, 31)
               for z in (0, 31) for t in (0, 63)]
    sites = np.unique(np.concatenate([rng.integers(0, V, 512), corners]))
    want = oracle.mop_sites(U, psi, dims, kappa, sites)
    gu.assert_close(got[sites], want, gu.TOL[prec], "32^3x64 sampled")
    del G, P, out
    torch.cuda.empty_cache()
