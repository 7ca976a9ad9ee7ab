"""Python binding of ``libwilson.so`` (the C ABI declared in include/wilson.h).

Argument marshalling only: every step of the computation runs in the HIP
library. torch tensors serve as device buffers and torch streams as HIP
streams. Packed fields are plain ``torch.uint8`` tensors of the byte size the
library reports; the layout is the library's even-odd layout (wilson.h).

Importing this module raises if the library is not built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwilson.so")

# flags (wilson.h)
F64 = 0x0
F32 = 0x1
F16S = 0x2
LINK18 = 0x0
LINK12 = 0x4
DAG = 0x8
HOP = 0x10
EO = 0x20
MIXED = 0x40
X0 = 0x80
GRAPH = 0x100
CANON = 0x200   # solvers: canonical complex128 gauge field and spinors (packed inside)

OK, NOCONV, BREAKDOWN, STAGNATED = 0, 1, 2, 3
EINVAL, EWORKSPACE, EHIP = -1, -2, -3
STATUS_NAMES = {0: "OK", 1: "NOCONV", 2: "BREAKDOWN", 3: "STAGNATED",
                -1: "EINVAL", -2: "EWORKSPACE", -3: "EHIP"}

ANTIPERIODIC_T = (1.0, 1.0, 1.0, -1.0)

# exported symbols, in the order of wilson.h
SYMBOLS = ("wl_version", "wl_last_error", "wl_spinor_bytes", "wl_gauge_bytes",
           "wl_pack_gauge", "wl_pack_spinor", "wl_unpack_spinor",
           "wilson_dslash", "wilson_dslash_eo", "wl_workspace_bytes",
           "solve_cg", "solve_bicgstab", "wilson_dslash_batch", "solve_cg_batch",
           "wl_problems_workspace_bytes", "solve_cg_problems",
           "wl_server_create", "wl_server_submit", "wl_server_wait", "wl_server_next",
           "wl_server_pending", "wl_server_destroy", "wl_tuning_report", "wl_stream_copy",
           "solve_cg_noalloc", "wilson_dslash_tm", "wilson_dslash_eo_tm", "solve_cg_tm",
           "solve_bicgstab_tm", "wl_meson_workspace_bytes", "wl_meson_correlators",
           "wl_heatbath", "wl_plaquette_workspace_bytes", "wl_plaquette",
           "wl_heatbath_packed", "wl_plaquette_packed", "wl_unpack_gauge")


class WilsonError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("true_res", ctypes.c_double), ("seconds", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("fp64_iterations", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class ServerConfig(ctypes.Structure):
    """The C struct wl_server_config."""
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("slots", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tol", ctypes.c_double),
                ("maxiter", ctypes.c_int32), ("phases", ctypes.c_double * 8),
                ("merge", ctypes.c_int32), ("site_slack", ctypes.c_double)]


class RequestTimes(ctypes.Structure):
    """The C struct wl_request_times (seconds since the server was created)."""
    _fields_ = [("submitted", ctypes.c_double), ("admitted", ctypes.c_double),
                ("finished", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwilson.so is not built (%s); run "
                          "`python -m paper_1112_5280_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, I32, D, SZ = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32,
                          ctypes.c_double, ctypes.c_size_t)
    lib.wl_version.restype = ctypes.c_char_p
    lib.wl_last_error.restype = ctypes.c_char_p
    lib.wl_spinor_bytes.argtypes = [P, U32, I32]
    lib.wl_spinor_bytes.restype = SZ
    lib.wl_gauge_bytes.argtypes = [P, U32]
    lib.wl_gauge_bytes.restype = SZ
    for f in (lib.wl_pack_gauge, lib.wl_pack_spinor, lib.wl_unpack_spinor, lib.wl_unpack_gauge):
        f.argtypes = [P, P, P, U32, P]
        f.restype = ctypes.c_int
    lib.wilson_dslash.argtypes = [P, P, P, P, D, P, U32, P]
    lib.wilson_dslash.restype = ctypes.c_int
    lib.wilson_dslash_eo.argtypes = [P, P, P, P, D, P, I32, U32, P]
    lib.wilson_dslash_eo.restype = ctypes.c_int
    lib.wl_workspace_bytes.argtypes = [P, U32, I32]
    lib.wl_workspace_bytes.restype = SZ
    for f in (lib.solve_cg, lib.solve_bicgstab):
        f.argtypes = [P, P, P, P, D, P, D, I32, U32, P, SZ,
                      ctypes.POINTER(SolveStats), P]
        f.restype = ctypes.c_int
    lib.wilson_dslash_tm.argtypes = [P, P, P, P, D, D, P, U32, P]
    lib.wilson_dslash_tm.restype = ctypes.c_int
    lib.wilson_dslash_eo_tm.argtypes = [P, P, P, P, D, D, P, I32, U32, P]
    lib.wilson_dslash_eo_tm.restype = ctypes.c_int
    for f in (lib.solve_cg_tm, lib.solve_bicgstab_tm):
        f.argtypes = [P, P, P, P, D, D, P, D, I32, U32, P, SZ, ctypes.POINTER(SolveStats), P]
        f.restype = ctypes.c_int
    for f in (lib.wl_heatbath, lib.wl_heatbath_packed):
        f.argtypes = [P, P, D, I32, U32, U32, P]
        f.restype = ctypes.c_int
    lib.wl_plaquette_workspace_bytes.argtypes = [P]
    lib.wl_plaquette_workspace_bytes.restype = SZ
    for f in (lib.wl_plaquette, lib.wl_plaquette_packed):
        f.argtypes = [P, P, P, P, SZ, P]
        f.restype = ctypes.c_int
    lib.wl_meson_workspace_bytes.argtypes = [P]
    lib.wl_meson_workspace_bytes.restype = SZ
    lib.wl_meson_correlators.argtypes = [P, P, I32, P, P, SZ, P]
    lib.wl_meson_correlators.restype = ctypes.c_int
    lib.solve_cg_noalloc.argtypes = [P, P, P, P, D, P, D, I32, U32,
                                     ctypes.POINTER(SolveStats), P]
    lib.solve_cg_noalloc.restype = ctypes.c_int
    lib.wilson_dslash_batch.argtypes = [P, P, P, I32, P, D, P, U32, P]
    lib.wilson_dslash_batch.restype = ctypes.c_int
    lib.solve_cg_batch.argtypes = [P, P, P, I32, P, D, P, D, I32, U32, P, SZ,
                                   ctypes.POINTER(SolveStats), P]
    lib.solve_cg_batch.restype = ctypes.c_int
    lib.wl_problems_workspace_bytes.argtypes = [P, I32, U32]
    lib.wl_problems_workspace_bytes.restype = SZ
    lib.solve_cg_problems.argtypes = [P, I32, P, D, I32, U32, P, SZ,
                                      ctypes.POINTER(SolveStats), P]
    lib.solve_cg_problems.restype = ctypes.c_int
    lib.wl_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
    lib.wl_server_create.restype = ctypes.c_int
    lib.wl_server_submit.argtypes = [P, P, ctypes.POINTER(ctypes.c_uint64)]
    lib.wl_server_submit.restype = ctypes.c_int
    lib.wl_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(SolveStats),
                                   ctypes.POINTER(RequestTimes)]
    lib.wl_server_wait.restype = ctypes.c_int
    lib.wl_server_next.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(SolveStats),
                                   ctypes.POINTER(RequestTimes)]
    lib.wl_server_next.restype = ctypes.c_int
    lib.wl_server_pending.argtypes = [P]
    lib.wl_server_pending.restype = I32
    lib.wl_server_destroy.argtypes = [P]
    lib.wl_server_destroy.restype = ctypes.c_int
    lib.wl_tuning_report.argtypes = [ctypes.c_char_p, SZ]
    lib.wl_tuning_report.restype = SZ
    lib.wl_stream_copy.argtypes = [P, P, SZ, P]
    lib.wl_stream_copy.restype = ctypes.c_int
    return lib


lib = _load()


# ---------------------------------------------------------------------------
def _dims(dims):
    return (ctypes.c_int32 * 4)(*[int(d) for d in dims])


def _phases(phases):
    ph = np.asarray(phases, dtype=np.complex128).reshape(4)
    flat = np.stack([ph.real, ph.imag], axis=1).reshape(-1)
    return (ctypes.c_double * 8)(*flat.tolist())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if t.device.type != "cuda":
            # every buffer of the ABI is device memory: a host pointer would
            # reach a kernel and fault the GPU
            raise ValueError("a device tensor is required, got one on %s" % t.device)
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


def _stream(stream, *keep):
    """The HIP stream of a library call: the current stream, or `stream`. A
    call on another stream than the current one is first ordered after the
    work already queued on the current stream (the producers of its inputs,
    and the last users of the memory the caching allocator just handed this
    binding there); the tensors in `keep`, allocated here, stay reserved until
    `stream` has passed the call."""
    cur = torch.cuda.current_stream()
    if stream is None:
        return ctypes.c_void_p(cur.cuda_stream)
    if stream != cur:
        stream.wait_stream(cur)
        for t in keep:
            if t is not None:
                t.record_stream(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _check(code, what):
    if code < 0:
        raise WilsonError(code, "%s: %s" % (what, last_error()))
    return code


def version() -> str:
    return lib.wl_version().decode()


def last_error() -> str:
    return lib.wl_last_error().decode()


def spinor_bytes(dims, flags=F64, nparity=2) -> int:
    n = lib.wl_spinor_bytes(_dims(dims), flags, nparity)
    if n == 0:
        raise WilsonError(EINVAL, "invalid dims/flags for a spinor: %s" % (dims,))
    return int(n)


def gauge_bytes(dims, flags=F64) -> int:
    n = lib.wl_gauge_bytes(_dims(dims), flags)
    if n == 0:
        raise WilsonError(EINVAL, "invalid dims/flags for a gauge field: %s" % (dims,))
    return int(n)


def workspace_bytes(dims, flags=F64, nrhs=1) -> int:
    return int(lib.wl_workspace_bytes(_dims(dims), flags, nrhs))


def empty_spinor(dims, flags=F64, nparity=2, device="cuda"):
    return torch.empty(spinor_bytes(dims, flags, nparity), dtype=torch.uint8, device=device)


def zeros_spinor(dims, flags=F64, nparity=2, device="cuda"):
    return torch.zeros(spinor_bytes(dims, flags, nparity), dtype=torch.uint8, device=device)


def parity_block(packed, dims, flags, parity):
    """View of one parity block (a half field) of a packed full spinor."""
    n = spinor_bytes(dims, flags, 1)
    return packed[parity * n:(parity + 1) * n]


def _canon_device(a, shape, device):
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
    a = a.to(device=device, dtype=torch.complex128).contiguous()
    if tuple(a.shape) != shape:
        raise ValueError("expected shape %s, got %s" % (shape, tuple(a.shape)))
    return a


def pack_gauge(U, dims, flags=F64, out=None, stream=None, device="cuda"):
    """Canonical complex128 U[V,4,3,3] (numpy or torch) -> packed device field."""
    V = int(np.prod(dims))
    Ud = _canon_device(U, (V, 4, 3, 3), device)
    if out is None:
        out = torch.empty(gauge_bytes(dims, flags), dtype=torch.uint8, device=device)
    _check(lib.wl_pack_gauge(_ptr(Ud), _ptr(out), _dims(dims), flags, _stream(stream, Ud, out)),
           "wl_pack_gauge")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return out


def pack_spinor(psi, dims, flags=F64, out=None, stream=None, device="cuda"):
    """Canonical complex128 psi[V,4,3] (numpy or torch) -> packed full spinor."""
    V = int(np.prod(dims))
    pd = _canon_device(psi, (V, 4, 3), device)
    if out is None:
        out = torch.empty(spinor_bytes(dims, flags, 2), dtype=torch.uint8, device=device)
    _check(lib.wl_pack_spinor(_ptr(pd), _ptr(out), _dims(dims), flags, _stream(stream, pd, out)),
           "wl_pack_spinor")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return out


def unpack_gauge(packed, dims, flags=F64, stream=None):
    """Packed gauge field -> canonical complex128 torch tensor [V,4,3,3] on device
    (the inverse of pack_gauge; 12-real fields get their third rows rebuilt)."""
    V = int(np.prod(dims))
    out = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device=packed.device)
    _check(lib.wl_unpack_gauge(_ptr(packed), _ptr(out), _dims(dims), flags,
                               _stream(stream, out)), "wl_unpack_gauge")
    return out


def unpack_spinor(packed, dims, flags=F64, stream=None):
    """Packed full spinor -> canonical complex128 torch tensor [V,4,3] on device."""
    V = int(np.prod(dims))
    out = torch.empty((V, 4, 3), dtype=torch.complex128, device=packed.device)
    _check(lib.wl_unpack_spinor(_ptr(packed), _ptr(out), _dims(dims), flags,
                                _stream(stream, out)), "wl_unpack_spinor")
    return out


def wilson_dslash(gauge, inp, out, dims, kappa, phases=ANTIPERIODIC_T, flags=F64,
                  stream=None):
    """out = M in (default), D_W in (HOP), or the adjoint (DAG); asynchronous."""
    return _check(lib.wilson_dslash(_ptr(gauge), _ptr(inp), _ptr(out), _dims(dims),
                                    float(kappa), _phases(phases), flags, _stream(stream)),
                  "wilson_dslash")


def wilson_dslash_eo(gauge, inp, out, dims, kappa, out_parity, phases=ANTIPERIODIC_T,
                     flags=F64, stream=None):
    """HOP: out_p = D_{p,1-p} in_{1-p} (half fields). Default: the Schur operator,
    in_p a half field and out a FULL field whose parity-p block receives
    Mhat_p in_p and whose other block receives the intermediate D_{1-p,p} in_p."""
    return _check(lib.wilson_dslash_eo(_ptr(gauge), _ptr(inp), _ptr(out), _dims(dims),
                                       float(kappa), _phases(phases), int(out_parity),
                                       flags, _stream(stream)), "wilson_dslash_eo")


def _solve(fn, name, gauge, b, x, dims, kappa, phases, tol, maxiter, flags, work, stream,
           mu=None):
    need = workspace_bytes(dims, flags)
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=b.device)
    st = SolveStats()
    extra = () if mu is None else (float(mu),)
    code = fn(_ptr(gauge), _ptr(b), _ptr(x), _dims(dims), float(kappa), *extra, _phases(phases),
              float(tol), int(maxiter), flags, _ptr(work), work.numel(), ctypes.byref(st),
              _stream(stream, work))
    _check(code, name)
    d = st.as_dict()
    d["status_name"] = STATUS_NAMES.get(code, "?")
    if code != OK:
        d["message"] = last_error()
    return d


def solve_cg(gauge, b, x, dims, kappa, phases=ANTIPERIODIC_T, tol=1e-10, maxiter=100000,
             flags=F64, work=None, stream=None):
    """CGNR solve of M x = b (packed FP64 b, x); returns the stats dict."""
    return _solve(lib.solve_cg, "solve_cg", gauge, b, x, dims, kappa, phases, tol, maxiter,
                  flags, work, stream)


def solve_bicgstab(gauge, b, x, dims, kappa, phases=ANTIPERIODIC_T, tol=1e-10,
                   maxiter=100000, flags=F64, work=None, stream=None):
    """BiCGStab solve of M x = b (packed FP64 b, x); returns the stats dict."""
    return _solve(lib.solve_bicgstab, "solve_bicgstab", gauge, b, x, dims, kappa, phases,
                  tol, maxiter, flags, work, stream)


def solve_cg_noalloc(gauge, b, x, dims, kappa, phases=ANTIPERIODIC_T, tol=1e-10,
                     maxiter=100000, flags=F64, stream=None):
    """solve_cg with the library's static scratch instead of a workspace: the
    call allocates nothing (lattices whose workspace fits in 64 MiB)."""
    st = SolveStats()
    code = lib.solve_cg_noalloc(_ptr(gauge), _ptr(b), _ptr(x), _dims(dims), float(kappa),
                                _phases(phases), float(tol), int(maxiter), flags,
                                ctypes.byref(st), _stream(stream))
    _check(code, "solve_cg_noalloc")
    d = st.as_dict()
    d["status_name"] = STATUS_NAMES.get(code, "?")
    if code != OK:
        d["message"] = last_error()
    return d


def wilson_dslash_tm(gauge, inp, out, dims, kappa, mu, phases=ANTIPERIODIC_T, flags=F64,
                     stream=None):
    """Twisted-mass operator M(mu) (or M(mu)^dag, or D_W with HOP); asynchronous."""
    return _check(lib.wilson_dslash_tm(_ptr(gauge), _ptr(inp), _ptr(out), _dims(dims),
                                       float(kappa), float(mu), _phases(phases), flags,
                                       _stream(stream)), "wilson_dslash_tm")


def wilson_dslash_eo_tm(gauge, inp, out, dims, kappa, mu, out_parity, phases=ANTIPERIODIC_T,
                        flags=F64, stream=None):
    """Twisted-mass even-odd operator: HOP as wilson_dslash_eo; default the Schur
    complement A - kappa^2 D A^-1 D into the parity-p block of the full field out."""
    return _check(lib.wilson_dslash_eo_tm(_ptr(gauge), _ptr(inp), _ptr(out), _dims(dims),
                                          float(kappa), float(mu), _phases(phases),
                                          int(out_parity), flags, _stream(stream)),
                  "wilson_dslash_eo_tm")


def solve_cg_tm(gauge, b, x, dims, kappa, mu, phases=ANTIPERIODIC_T, tol=1e-10,
                maxiter=100000, flags=F64, work=None, stream=None):
    """CGNR solve of M(mu) x = b (twisted mass); returns the stats dict."""
    return _solve(lib.solve_cg_tm, "solve_cg_tm", gauge, b, x, dims, kappa, phases, tol,
                  maxiter, flags, work, stream, mu=mu)


def solve_bicgstab_tm(gauge, b, x, dims, kappa, mu, phases=ANTIPERIODIC_T, tol=1e-10,
                      maxiter=100000, flags=F64, work=None, stream=None):
    """BiCGStab solve of M(mu) x = b (twisted mass); returns the stats dict."""
    return _solve(lib.solve_bicgstab_tm, "solve_bicgstab_tm", gauge, b, x, dims, kappa,
                  phases, tol, maxiter, flags, work, stream, mu=mu)


def meson_correlators(props, dims, t0=0, work=None, stream=None):
    """Eq. 1's C_Gamma(t) for the 16 Gamma_n from 12 propagator columns (a batch
    of packed FP64 full spinors, field 3 b + c); returns a complex128 tensor
    [16, Lt] on the device (t counted from t0)."""
    Lt = int(dims[3])
    corr = torch.empty((16, Lt, 2), dtype=torch.float64, device=props.device)
    if work is None:
        work = torch.empty(max(int(lib.wl_meson_workspace_bytes(_dims(dims))), 1),
                           dtype=torch.uint8, device=props.device)
    _check(lib.wl_meson_correlators(_ptr(props), _dims(dims), int(t0), _ptr(corr), _ptr(work),
                                    work.numel(), _stream(stream, corr, work)),
           "wl_meson_correlators")
    return torch.view_as_complex(corr)


def heatbath(U, dims, beta, nsweeps=1, sweep0=0, seed=0, stream=None):
    """nsweeps SU(3) heat-bath sweeps in place on the canonical complex128 field
    U[V, 4, 3, 3] (a contiguous device tensor); asynchronous."""
    V = int(np.prod(dims))
    if (not isinstance(U, torch.Tensor) or U.dtype != torch.complex128 or not U.is_contiguous()
            or tuple(U.shape) != (V, 4, 3, 3)):
        raise ValueError("U must be a contiguous complex128 device tensor [V, 4, 3, 3]")
    _check(lib.wl_heatbath(_ptr(U), _dims(dims), float(beta), int(nsweeps),
                           int(sweep0) & 0xffffffff, int(seed) & 0xffffffff, _stream(stream)),
           "wl_heatbath")


def plaquette(U, dims, stream=None):
    """Mean plaquette of the canonical complex128 device field U[V, 4, 3, 3]."""
    return _plaquette(lib.wl_plaquette, "wl_plaquette", U, dims, stream)


def _packed_field(G, dims):
    if (not isinstance(G, torch.Tensor) or G.dtype != torch.uint8 or not G.is_contiguous()
            or G.numel() != gauge_bytes(dims, F64)):
        raise ValueError("G must be the packed FP64 18-real field (pack_gauge(U, dims, F64))")


def heatbath_packed(G, dims, beta, nsweeps=1, sweep0=0, seed=0, stream=None):
    """heatbath on the packed FP64 18-real field G (pack_gauge(U, dims)): the
    same update as heatbath on U, with coalesced loads; asynchronous."""
    _packed_field(G, dims)
    _check(lib.wl_heatbath_packed(_ptr(G), _dims(dims), float(beta), int(nsweeps),
                                  int(sweep0) & 0xffffffff, int(seed) & 0xffffffff,
                                  _stream(stream)), "wl_heatbath_packed")


def plaquette_packed(G, dims, stream=None):
    """Mean plaquette of the packed FP64 18-real field G."""
    _packed_field(G, dims)
    return _plaquette(lib.wl_plaquette_packed, "wl_plaquette_packed", G, dims, stream)


def _plaquette(fn, name, field, dims, stream):
    out = torch.empty(1, dtype=torch.float64, device=field.device)
    work = torch.empty(max(int(lib.wl_plaquette_workspace_bytes(_dims(dims))), 8),
                       dtype=torch.uint8, device=field.device)
    _check(fn(_ptr(field), _dims(dims), _ptr(out), _ptr(work), work.numel(),
              _stream(stream, out, work)), name)
    (torch.cuda.current_stream() if stream is None else stream).synchronize()
    return float(out.cpu())


def empty_batch(dims, nrhs, flags=F64, device="cuda"):
    """nrhs packed full spinors stored one after another."""
    return torch.empty(nrhs * spinor_bytes(dims, flags, 2), dtype=torch.uint8, device=device)


def batch_field(batch, dims, flags, r):
    """View of field r of a batch."""
    n = spinor_bytes(dims, flags, 2)
    return batch[r * n:(r + 1) * n]


def wilson_dslash_batch(gauge, inp, out, nrhs, dims, kappa, phases=ANTIPERIODIC_T,
                        flags=F64, stream=None):
    """The operator of wilson_dslash on nrhs fields stored one after another."""
    return _check(lib.wilson_dslash_batch(_ptr(gauge), _ptr(inp), _ptr(out), int(nrhs),
                                          _dims(dims), float(kappa), _phases(phases), flags,
                                          _stream(stream)), "wilson_dslash_batch")


def solve_cg_batch(gauge, b, x, nrhs, dims, kappa, phases=ANTIPERIODIC_T, tol=1e-10,
                   maxiter=100000, flags=F64, work=None, stream=None):
    """Batched CGNR of nrhs right-hand sides; returns (status, [stats per RHS])."""
    need = workspace_bytes(dims, flags, nrhs)
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=b.device)
    st = (SolveStats * int(nrhs))()
    code = lib.solve_cg_batch(_ptr(gauge), _ptr(b), _ptr(x), int(nrhs), _dims(dims),
                              float(kappa), _phases(phases), float(tol), int(maxiter), flags,
                              _ptr(work), work.numel(), st, _stream(stream, work))
    _check(code, "solve_cg_batch")
    out = []
    for s in st:
        d = s.as_dict()
        d["status_name"] = STATUS_NAMES.get(d["status"], "?")
        out.append(d)
    return code, out


class ProblemDesc(ctypes.Structure):
    """The C struct wl_problem."""
    _fields_ = [("dims", ctypes.c_int32 * 4), ("kappa", ctypes.c_double),
                ("gauge", ctypes.c_void_p), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


@dataclass
class Problem:
    """One problem of an uneven batch: packed FP64 gauge field, source and solution
    (full lattice, packed layout) resident on the device."""
    dims: tuple
    kappa: float
    gauge: torch.Tensor
    b: torch.Tensor
    x: torch.Tensor


def _problem_array(problems):
    arr = (ProblemDesc * len(problems))()
    for i, q in enumerate(problems):
        arr[i].dims = _dims(q.dims)
        arr[i].kappa = float(q.kappa)
        arr[i].gauge = q.gauge.data_ptr()
        arr[i].b = q.b.data_ptr()
        arr[i].x = q.x.data_ptr()
    return arr


def problems_workspace_bytes(problems, flags=F64):
    arr = _problem_array(problems)
    return lib.wl_problems_workspace_bytes(arr, len(problems), flags)


def solve_cg_problems(problems, phases=ANTIPERIODIC_T, tol=1e-10, maxiter=100000, flags=F64,
                      work=None, stream=None):
    """CGNR over an uneven batch of independent problems (sizes, kappas and gauge
    fields may all differ); returns (status, [stats per problem])."""
    arr = _problem_array(problems)
    n = len(problems)
    need = lib.wl_problems_workspace_bytes(arr, n, flags)
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=problems[0].b.device)
    st = (SolveStats * n)()
    code = lib.solve_cg_problems(arr, n, _phases(phases), float(tol), int(maxiter), flags,
                                 _ptr(work), work.numel(), st, _stream(stream, work))
    _check(code, "solve_cg_problems")
    out = []
    for s in st:
        d = s.as_dict()
        d["status_name"] = STATUS_NAMES.get(d["status"], "?")
        out.append(d)
    return code, out


def stream_copy(src, dst, nbytes=None, stream=None):
    """Streaming device copy (the achievable-bandwidth reference)."""
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    _check(lib.wl_stream_copy(_ptr(src), _ptr(dst), n, _stream(stream)), "wl_stream_copy")


def tuning_report():
    """The autotuner's record: one line per tuned batched-operator shape."""
    n = lib.wl_tuning_report(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib.wl_tuning_report(buf, n + 1)
    return buf.value.decode()


class Server:
    """A solve server (wl_server_*): requests of any lattice size are admitted
    as solve slots and HBM-budget memory free up, earliest deadline first (the
    deadline: submission time plus site_slack seconds per lattice site; 0 is
    first-in first-out), and the admitted solves run concurrently, one stream
    per slot. With merge > 1 a slot also takes up to merge - 1 more waiting
    requests of the same lattice size and solves them as one batch (results
    bitwise those of solo solves).

    The caller keeps each request's gauge, b and x tensors alive until the
    request is collected with wait() or next()."""

    def __init__(self, hbm_budget, slots=4, flags=EO | MIXED, tol=1e-10, maxiter=100000,
                 phases=ANTIPERIODIC_T, merge=1, site_slack=0.0):
        cfg = ServerConfig()
        cfg.merge = int(merge)
        cfg.site_slack = float(site_slack)
        cfg.hbm_budget = int(hbm_budget)
        cfg.slots = int(slots)
        cfg.flags = int(flags)
        cfg.tol = float(tol)
        cfg.maxiter = int(maxiter)
        cfg.phases = _phases(phases)
        h = ctypes.c_void_p()
        _check(lib.wl_server_create(ctypes.byref(cfg), ctypes.byref(h)), "wl_server_create")
        self._h = h
        self.flags = flags
        self._keep = {}

    def submit(self, problem):
        """Queue one Problem (its x receives the solution); returns the ticket."""
        d = ProblemDesc()
        d.dims = _dims(problem.dims)
        d.kappa = float(problem.kappa)
        d.gauge = problem.gauge.data_ptr()
        d.b = problem.b.data_ptr()
        d.x = problem.x.data_ptr()
        t = ctypes.c_uint64()
        _check(lib.wl_server_submit(self._h, ctypes.byref(d), ctypes.byref(t)), "wl_server_submit")
        self._keep[t.value] = problem
        return t.value

    def _result(self, code, ticket, st, tm):
        _check(code, "wl_server")
        self._keep.pop(ticket, None)
        d = st.as_dict()
        d["status_name"] = STATUS_NAMES.get(d["status"], "?")
        return code, d, tm.as_dict()

    def wait(self, ticket):
        """Block until `ticket` finishes; returns (status, stats, times)."""
        st, tm = SolveStats(), RequestTimes()
        code = lib.wl_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(tm))
        return self._result(code, ticket, st, tm)

    def next(self):
        """Block until any uncollected request finishes; returns
        (ticket, status, stats, times)."""
        st, tm, t = SolveStats(), RequestTimes(), ctypes.c_uint64()
        code = lib.wl_server_next(self._h, ctypes.byref(t), ctypes.byref(st), ctypes.byref(tm))
        return (t.value,) + self._result(code, t.value, st, tm)

    def pending(self):
        return lib.wl_server_pending(self._h)

    def close(self):
        if self._h is not None:
            code = lib.wl_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            _check(code, "wl_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
