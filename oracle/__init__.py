"""FP64 CPU oracle of the Wilson-Dirac operator and its Krylov solves.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``. The product path (the HIP
library ``libwilson.so`` and its binding in ``paper_1112_5280_amd``) never
imports, links or runs anything here, and nothing here imports the product.

The arithmetic lives in ``wilson_oracle.c`` (plain C, FP64, OpenMP over sites);
this module compiles it with gcc on first use and marshals numpy arrays.
Canonical layouts: ``U[V,4,3,3]`` and ``psi[V,4,3]`` complex128, site index
``x + Lx*(y + Ly*(z + Lz*t))``; ``phases`` are the 4 complex boundary phases
(forward hops that wrap pick up ``phase_mu``, backward ones its conjugate).

Parity status of each function is recorded in ``PINS`` below and in the tests
that pin it (``tests/test_oracle_pins.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson_oracle.c")
_LIB = os.path.join(_HERE, "libwilson_oracle.so")
_lock = threading.Lock()
_lib = None

ANTIPERIODIC_T = (1.0, 1.0, 1.0, -1.0)

# Which independent fact pins each oracle function (see tests/test_oracle_pins.py)
PINS = {
    "dslash/mop": "free-field plane-wave eigenvalues (closed form), dense "
                  "Kronecker-assembled operator on 2^4 and 2x4x2x4, gauge "
                  "covariance, gamma5-hermiticity",
    "mop dagger": "adjoint identity <phi, M psi> = <M^dag phi, psi>",
    "dslash_eo/schur": "D_W = D_eo + D_oe split; Schur complement vs dense "
                       "block elimination",
    "cgnr/bicgstab": "LAPACK dense solve on 4^4; Neumann series for "
                     "kappa < 1/8; free-field plane-wave source",
    "mop_tm/cgnr_tm": "free-field eigenvalues 1 - 2k sum cos p +- 2ik sqrt(mu^2 + "
                      "sum sin^2 p); g5 M(mu) g5 = M(-mu)^dag; mu = 0 is M; dense "
                      "2x4x2x4 with the twist; LAPACK solve",
    "philox/kp_samples/heatbath": "Philox4x32-10 known-answer vectors; the Kennedy-"
                                  "Pendleton density (mean I_2/I_1, KS test); SU(3) kept; "
                                  "strong-coupling beta/18 and weak-coupling 1 - 2/beta",
    "meson": "pion channel -sum |S|^2; completeness of the 16 Gammas "
             "(sum_n Gamma_n^2 C_n = -4 sum |Tr_spin S|^2); gauge invariance; time shift",
    "cgnr_eo": "LAPACK dense solve on 4^4 and 2x4x2x4; the odd rows of M x = b "
               "hold exactly; free-field plane-wave source",
    "plaquette": "unit links give 1; gauge invariance",
    "singular_extremes": "LAPACK singular values of the dense operator on "
                         "2x4x2x4; free-field closed form min/max |lambda(p)|",
}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -O2, OpenMP, no fast-math)."""
    with _lock:
        if force or not os.path.exists(_LIB) or \
                os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                   "-Wall", _SRC, "-o", tmp, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
    return _LIB


class OrcStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("true_res", ctypes.c_double)]


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (4,) or (d < 1).any():
        raise ValueError("dims must be 4 positive extents")
    return d


def _phases(phases):
    return np.ascontiguousarray(np.asarray(phases, dtype=np.complex128).reshape(4))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _vol(d):
    return int(np.prod(d.astype(np.int64)))


class Oracle:
    """The oracle's functions bound to one compiled copy of ``wilson_oracle.c``.

    The module-level functions use the default copy; tests that plant
    mistakes in a copy of the source bind an ``Oracle`` to that build.
    """

    def __init__(self, path):
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.orc_gamma.argtypes = [I, P]
        lib.orc_max_threads.restype = I
        lib.orc_set_threads.argtypes = [I]
        lib.orc_dslash.argtypes = [P, P, P, P, P, I]
        lib.orc_mop.argtypes = [P, P, P, P, P, D, I]
        lib.orc_mop_tm.argtypes = [P, P, P, P, P, D, D, I]
        lib.orc_schur_tm.argtypes = [P, P, P, P, P, D, D, I, I]
        lib.orc_cgnr_tm.argtypes = [P, P, P, P, P, D, D, D, I, ctypes.POINTER(OrcStats)]
        lib.orc_cgnr_tm.restype = I
        lib.orc_mop_sites.argtypes = [P, P, P, P, D, I, P, ctypes.c_long, P]
        lib.orc_dslash_sites.argtypes = [P, P, P, P, I, P, ctypes.c_long, P]
        lib.orc_dslash_eo.argtypes = [P, P, P, P, P, I, I]
        lib.orc_schur.argtypes = [P, P, P, P, P, D, I, I]
        lib.orc_lanczos_mdm.argtypes = [P, P, P, P, D, I, P, P]
        lib.orc_lanczos_mdm.restype = I
        lib.orc_meson.argtypes = [P, P, I, P]
        lib.orc_philox.argtypes = [P, P, P]
        lib.orc_kp_samples.argtypes = [D, I, ctypes.c_uint32, P]
        lib.orc_heatbath.argtypes = [P, P, D, I, ctypes.c_uint32, ctypes.c_uint32]
        lib.orc_plaquette.argtypes = [P, P]
        lib.orc_plaquette.restype = D
        for fn in (lib.orc_cgnr, lib.orc_cgnr_eo, lib.orc_bicgstab):
            fn.argtypes = [P, P, P, P, P, D, D, I, ctypes.POINTER(OrcStats)]
            fn.restype = I
        self.lib = lib
        self.path = path

    def set_threads(self, n: int) -> None:
        self.lib.orc_set_threads(int(n))

    def max_threads(self) -> int:
        return int(self.lib.orc_max_threads())

    def gamma(self, mu: int) -> np.ndarray:
        """The oracle's Dirac matrix gamma_mu (mu=0..3) or gamma_5 (mu=4)."""
        out = np.zeros((4, 4, 2))
        self.lib.orc_gamma(int(mu), _ptr(out))
        return out[..., 0] + 1j * out[..., 1]

    def _fields(self, U, psi, dims):
        d = _dims(dims)
        v = _vol(d)
        return d, _c128(U, (v, 4, 3, 3)), _c128(psi, (v, 4, 3))

    def dslash(self, U, psi, dims, phases=ANTIPERIODIC_T, dagger=False):
        """D_W psi (the hopping term); ``dagger`` gives g5 D_W g5 = D_W^dag."""
        d, U, psi = self._fields(U, psi, dims)
        out = np.empty_like(psi)
        ph = _phases(phases)
        self.lib.orc_dslash(_ptr(U), _ptr(psi), _ptr(out), _ptr(d), _ptr(ph),
                            int(dagger))
        return out

    def mop(self, U, psi, dims, kappa, phases=ANTIPERIODIC_T, dagger=False):
        """M psi = psi - kappa D_W psi; ``dagger`` gives M^dag = g5 M g5."""
        d, U, psi = self._fields(U, psi, dims)
        out = np.empty_like(psi)
        ph = _phases(phases)
        self.lib.orc_mop(_ptr(U), _ptr(psi), _ptr(out), _ptr(d), _ptr(ph),
                         float(kappa), int(dagger))
        return out

    def mop_tm(self, U, psi, dims, kappa, mu, phases=ANTIPERIODIC_T, dagger=False):
        """Twisted-mass operator M(mu) psi = psi + 2 i kappa mu g5 psi - kappa D_W psi;
        ``dagger`` gives M(mu)^dag = g5 M(-mu) g5."""
        d, U, psi = self._fields(U, psi, dims)
        out = np.empty_like(psi)
        ph = _phases(phases)
        self.lib.orc_mop_tm(_ptr(U), _ptr(psi), _ptr(out), _ptr(d), _ptr(ph),
                            float(kappa), float(mu), int(dagger))
        return out

    def schur_tm(self, U, psi, dims, kappa, mu, parity=0, phases=ANTIPERIODIC_T,
                 dagger=False):
        """Twisted-mass Schur complement S_p psi = A psi - kappa^2 D_{p,1-p} A^-1
        D_{1-p,p} psi on parity p, A = 1 + 2 i kappa mu g5 (zero on parity 1-p)."""
        d, U, psi = self._fields(U, psi, dims)
        out = np.empty_like(psi)
        ph = _phases(phases)
        self.lib.orc_schur_tm(_ptr(U), _ptr(psi), _ptr(out), _ptr(d), _ptr(ph),
                              float(kappa), float(mu), int(parity), int(dagger))
        return out

    def cgnr_tm(self, U, b, dims, kappa, mu, tol=1e-10, maxiter=100000,
                phases=ANTIPERIODIC_T, x0=None):
        """Solve M(mu) x = b by CGNR; returns ``(x, stats)``."""
        d, U, b = self._fields(U, b, dims)
        x = np.zeros_like(b) if x0 is None else _c128(x0, b.shape).copy()
        ph = _phases(phases)
        st = OrcStats()
        status = self.lib.orc_cgnr_tm(_ptr(U), _ptr(b), _ptr(x), _ptr(d), _ptr(ph),
                                      float(kappa), float(mu), float(tol), int(maxiter),
                                      ctypes.byref(st))
        return x, dict(status=int(status), iterations=int(st.iterations),
                       restarts=int(st.restarts), true_res=float(st.true_res))

    def true_residual_tm(self, U, b, x, dims, kappa, mu, phases=ANTIPERIODIC_T):
        """||b - M(mu) x|| / ||b|| with the oracle's FP64 twisted-mass operator."""
        r = _c128(b) - self.mop_tm(U, x, dims, kappa, mu, phases)
        return float(np.linalg.norm(r) / np.linalg.norm(b))

    def _sites(self, sites, v):
        s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64).reshape(-1))
        if s.size and (s.min() < 0 or s.max() >= v):
            raise ValueError("site out of range")
        return s

    def mop_sites(self, U, psi, dims, kappa, sites, phases=ANTIPERIODIC_T,
                  dagger=False):
        """M psi at the listed sites only; returns ``[n, 4, 3]``."""
        d, U, psi = self._fields(U, psi, dims)
        s = self._sites(sites, _vol(d))
        out = np.empty((s.size, 4, 3), dtype=np.complex128)
        ph = _phases(phases)
        self.lib.orc_mop_sites(_ptr(U), _ptr(psi), _ptr(d), _ptr(ph),
                               float(kappa), int(dagger), _ptr(s), s.size,
                               _ptr(out))
        return out

    def dslash_sites(self, U, psi, dims, sites, phases=ANTIPERIODIC_T,
                     dagger=False):
        """D_W psi at the listed sites only; returns ``[n, 4, 3]``."""
        d, U, psi = self._fields(U, psi, dims)
        s = self._sites(sites, _vol(d))
        out = np.empty((s.size, 4, 3), dtype=np.complex128)
        ph = _phases(phases)
        self.lib.orc_dslash_sites(_ptr(U), _ptr(psi), _ptr(d), _ptr(ph),
                                  int(dagger), _ptr(s), s.size, _ptr(out))
        return out

    def dslash_eo(self, U, psi, dims, out_parity, phases=ANTIPERIODIC_T,
                  dagger=False):
        """D_{p,1-p}: output on parity ``out_parity`` from the other parity.

        Whole-lattice arrays in and out; the output is zero on parity 1-p.
        """
        d, U, psi = self._fields(U, psi, dims)
        out = np.empty_like(psi)
        ph = _phases(phases)
        self.lib.orc_dslash_eo(_ptr(U), _ptr(psi), _ptr(out), _ptr(d), _ptr(ph),
                               int(out_parity), int(dagger))
        return out

    def schur(self, U, psi, dims, kappa, parity=0, phases=ANTIPERIODIC_T,
              dagger=False):
        """Mhat_p psi = psi - kappa^2 D_{p,1-p} D_{1-p,p} psi on parity p."""
        d, U, psi = self._fields(U, psi, dims)
        out = np.empty_like(psi)
        ph = _phases(phases)
        self.lib.orc_schur(_ptr(U), _ptr(psi), _ptr(out), _ptr(d), _ptr(ph),
                           float(kappa), int(parity), int(dagger))
        return out

    def meson(self, props, dims, t0=0):
        """Meson correlators of Eq. 1, C_Gamma(t) = -sum_xvec Tr(S^dag g5 Gamma S
        Gamma g5), for the 16 Gamma_n = g_x^n0 g_y^n1 g_z^n2 g_t^n3 (bits of n),
        t counted from t0. ``props`` is [12, V, 4, 3]: the solutions for the
        point sources of spin b and colour c in row 3 b + c. Returns a complex
        array [16, Lt]."""
        d = _dims(dims)
        v = _vol(d)
        pr = _c128(props, (12, v, 4, 3))
        out = np.zeros((16, int(d[3])), dtype=np.complex128)
        self.lib.orc_meson(_ptr(pr), _ptr(d), int(t0), _ptr(out))
        return out

    def philox(self, ctr, key):
        """Philox4x32-10 of a 4-word counter and a 2-word key (four words)."""
        c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
        k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
        o = np.zeros(4, dtype=np.uint32)
        self.lib.orc_philox(_ptr(c), _ptr(k), _ptr(o))
        return [int(v) for v in o]

    def kp_samples(self, alpha, n, seed=0):
        """n Kennedy-Pendleton draws of x0 (density ~ sqrt(1 - x0^2) exp(alpha x0))."""
        out = np.zeros(int(n))
        self.lib.orc_kp_samples(float(alpha), int(n), int(seed) & 0xffffffff, _ptr(out))
        return out

    def heatbath(self, U, dims, beta, nsweeps, sweep0=0, seed=0):
        """nsweeps SU(3) heat-bath sweeps (Cabibbo-Marinari, Kennedy-Pendleton,
        Philox4x32-10 counters) in place on U [V, 4, 3, 3] (C-contiguous complex128)."""
        d = _dims(dims)
        if not (isinstance(U, np.ndarray) and U.dtype == np.complex128 and
                U.flags["C_CONTIGUOUS"] and U.shape == (_vol(d), 4, 3, 3)):
            raise ValueError("U must be a C-contiguous complex128 array [V, 4, 3, 3]")
        self.lib.orc_heatbath(_ptr(U), _ptr(d), float(beta), int(nsweeps),
                              int(sweep0) & 0xffffffff, int(seed) & 0xffffffff)
        return U

    def plaquette(self, U, dims) -> float:
        d = _dims(dims)
        U = _c128(U, (_vol(d), 4, 3, 3))
        return float(self.lib.orc_plaquette(_ptr(U), _ptr(d)))

    def _solve(self, fn, U, b, dims, kappa, tol, maxiter, phases, x0):
        d, U, b = self._fields(U, b, dims)
        x = np.zeros_like(b) if x0 is None else \
            _c128(x0, b.shape).copy()
        ph = _phases(phases)
        st = OrcStats()
        status = fn(_ptr(U), _ptr(b), _ptr(x), _ptr(d), _ptr(ph), float(kappa),
                    float(tol), int(maxiter), ctypes.byref(st))
        return x, dict(status=int(status), iterations=int(st.iterations),
                       restarts=int(st.restarts), true_res=float(st.true_res))

    def cgnr(self, U, b, dims, kappa, tol=1e-10, maxiter=100000,
             phases=ANTIPERIODIC_T, x0=None):
        """Solve M x = b by CG on M^dag M x = M^dag b; returns ``(x, stats)``."""
        return self._solve(self.lib.orc_cgnr, U, b, dims, kappa, tol, maxiter,
                           phases, x0)

    def cgnr_eo(self, U, b, dims, kappa, tol=1e-10, maxiter=100000,
                phases=ANTIPERIODIC_T, x0=None):
        """Solve M x = b by CG on the even-odd Schur system
        Mhat^dag Mhat x_e = Mhat^dag (b_e + kappa D_eo b_o), then
        x_o = b_o + kappa D_oe x_e; acceptance on the full residual.
        Returns ``(x, stats)``."""
        return self._solve(self.lib.orc_cgnr_eo, U, b, dims, kappa, tol, maxiter,
                           phases, x0)

    def bicgstab(self, U, b, dims, kappa, tol=1e-10, maxiter=100000,
                 phases=ANTIPERIODIC_T, x0=None):
        """Solve M x = b by BiCGStab on M; returns ``(x, stats)``."""
        return self._solve(self.lib.orc_bicgstab, U, b, dims, kappa, tol,
                           maxiter, phases, x0)

    def true_residual(self, U, b, x, dims, kappa, phases=ANTIPERIODIC_T):
        """||b - M x|| / ||b|| with the oracle's FP64 M."""
        r = _c128(b) - self.mop(U, x, dims, kappa, phases)
        return float(np.linalg.norm(r) / np.linalg.norm(b))

    def singular_extremes(self, U, dims, kappa, steps=300, seed=0,
                          phases=ANTIPERIODIC_T):
        """Largest and smallest singular value of M and cond(M) = their ratio.

        Two solutions whose true residuals are rho and rho* differ by at most
        cond(M) (rho + rho*) relative to the solution, so this condition number
        is the scale on which solutions from different solvers and precisions
        are compared. Plain Lanczos tridiagonalisation of A = M^dag M from a
        complex Gaussian start vector (``seed``); sigma^2 are the extreme
        eigenvalues of the ``steps`` x ``steps`` tridiagonal matrix. Without
        reorthogonalisation, lost orthogonality only repeats Ritz values that
        have converged; it does not move the extreme ones. The smallest Ritz
        value approaches lambda_min(A) from above, so until it has converged
        cond is an underestimate. Returns ``(sigma_max, sigma_min, cond)``.
        """
        d = _dims(dims)
        U = _c128(U, (_vol(d), 4, 3, 3))
        shape = (_vol(d), 4, 3)
        rng = np.random.default_rng(seed)
        v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        v = np.ascontiguousarray(v / np.linalg.norm(v))
        alpha = np.zeros(steps)
        beta = np.zeros(max(steps - 1, 1))
        ph = _phases(phases)
        k = int(self.lib.orc_lanczos_mdm(_ptr(U), _ptr(v), _ptr(d), _ptr(ph), float(kappa),
                                         int(steps), _ptr(alpha), _ptr(beta)))
        T = np.diag(alpha[:k]) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
        ev = np.linalg.eigvalsh(T)
        smax, smin = float(np.sqrt(ev[-1])), float(np.sqrt(max(ev[0], 0.0)))
        return smax, smin, smax / smin


def default() -> Oracle:
    """The oracle built from ``wilson_oracle.c`` (compiled on first use)."""
    global _lib
    if _lib is None:
        build()
        _lib = Oracle(_LIB)
    return _lib


def _forward(name):
    def f(*args, **kwargs):
        return getattr(default(), name)(*args, **kwargs)
    f.__name__ = name
    f.__doc__ = getattr(Oracle, name).__doc__
    return f


for _name in ("set_threads", "max_threads", "gamma", "dslash", "mop",
              "mop_sites", "dslash_sites", "dslash_eo", "schur", "plaquette",
              "cgnr", "cgnr_eo", "bicgstab", "mop_tm", "schur_tm", "cgnr_tm", "meson", "philox", "kp_samples",
              "heatbath", "true_residual_tm", "true_residual", "singular_extremes"):
    globals()[_name] = _forward(_name)


def compile_copy(src_text: str, out_path: str) -> str:
    """Compile a (possibly modified) copy of the oracle source to ``out_path``."""
    src = out_path[:-3] + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                    "-w", src, "-o", out_path, "-lm"], check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def parity_mask(dims) -> np.ndarray:
    """Boolean ``[V]``: True on odd sites ((x+y+z+t) odd)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                             np.arange(lx), indexing="ij")
    return ((x + y + z + t) % 2 == 1).reshape(-1)
