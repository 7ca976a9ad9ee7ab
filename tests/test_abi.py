"""The C-ABI library loads, exports every symbol include/wilson.h declares, and
its host-side argument checks work (no GPU needed: nothing here launches)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wilson.h")


@pytest.fixture(scope="module")
def w():
    from paper_1112_5280_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1112_5280_amd import wilson
    return wilson


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("wilson_dslash", "wilson_dslash_eo", "solve_cg", "solve_bicgstab"):
        assert n in names


def test_every_declared_symbol_is_exported(w):
    names = declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", w.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(w.SYMBOLS)
    for n in names:
        assert hasattr(w.lib, n)


def test_sizes(w):
    d = (4, 4, 4, 4)              # Vh = 128 = S
    assert w.spinor_bytes(d, w.F64, 1) == 128 * 12 * 16
    assert w.spinor_bytes(d, w.F32, 2) == 2 * 128 * 12 * 8
    assert w.gauge_bytes(d, w.F64) == 2 * 4 * 9 * 16 * 128
    assert w.gauge_bytes(d, w.F32 | w.LINK12) == 2 * 4 * 6 * 8 * 128
    d = (6, 4, 6, 10)             # Vh = 720 -> S = 768
    assert w.spinor_bytes(d, w.F64, 1) == 768 * 12 * 16
    assert w.workspace_bytes(d, w.MIXED) > w.workspace_bytes(d, 0) > 0
    assert w.lib.wl_spinor_bytes(w._dims((3, 4, 4, 4)), 0, 2) == 0
    assert w.lib.wl_gauge_bytes(w._dims((4, 4, 4, 4)), 0x3) == 0


def _p(v):
    return ctypes.c_void_p(v)


def test_argument_checks_return_einval(w):
    d, ph = w._dims((4, 4, 4, 4)), w._phases(w.ANTIPERIODIC_T)
    lib = w.lib
    assert lib.wilson_dslash(None, None, None, w._dims((4, 4, 4, 3)), 0.1, ph, 0, None) == -1
    assert "even" in w.last_error()
    assert lib.wilson_dslash(_p(8), _p(16), _p(16), d, 0.1, ph, 0, None) == -1
    assert "alias" in w.last_error()
    assert lib.wilson_dslash(_p(8), _p(16), _p(32), d, 0.1,
                             w._phases((1, 1, 1, 0.5)), 0, None) == -1
    assert lib.wilson_dslash(_p(8), _p(16), _p(32), d, float("nan"), ph, 0, None) == -1
    assert lib.wilson_dslash(_p(8), _p(16), _p(32), d, 0.1, ph, 1 << 20, None) == -1
    assert lib.wilson_dslash_eo(_p(8), _p(16), _p(32), d, 0.1, ph, 2, 0, None) == -1
    assert lib.wl_pack_spinor(_p(8), _p(8), d, 0, None) == -1


def test_solver_argument_checks(w):
    d, ph = w._dims((4, 4, 4, 4)), w._phases(w.ANTIPERIODIC_T)
    st = w.SolveStats()
    call = lambda **k: w.lib.solve_cg(
        _p(8), _p(16), _p(k.get("x", 24)), k.get("dims", d), 0.1, ph, k.get("tol", 1e-10),
        k.get("maxiter", 10), k.get("flags", 0), _p(32), k.get("work", 1 << 30),
        ctypes.byref(st), None)
    assert call(work=10) == -2 and "workspace" in w.last_error()
    assert call(x=16) == -1                       # b aliases x
    assert call(tol=0.0) == -1
    assert call(maxiter=0) == -1
    assert call(flags=w.F32) == -1                # solver buffers are FP64
    assert call(flags=w.DAG) == -1
    assert call(dims=w._dims((4, 4, 4, 5))) == -1


def test_problem_argument_checks(w):
    ph = w._phases(w.ANTIPERIODIC_T)
    arr = (w.ProblemDesc * 2)()
    for i, dims in enumerate(((4, 4, 4, 4), (4, 4, 4, 8))):
        arr[i].dims = w._dims(dims)
        arr[i].kappa = 0.12
        arr[i].gauge, arr[i].b, arr[i].x = 8, 16 + 64 * i, 24 + 64 * i
    st = (w.SolveStats * 2)()
    need = w.lib.wl_problems_workspace_bytes(arr, 2, 0)
    # two sizes make two groups
    assert need > w.lib.wl_problems_workspace_bytes(arr, 1, 0) > 0
    call = lambda n=2, flags=0, work=need, tol=1e-10: w.lib.solve_cg_problems(
        arr, n, ph, tol, 10, flags, _p(32), work, st, None)
    assert call(n=0) == -1
    assert call(work=need - 1) == -2 and "workspace" in w.last_error()
    assert call(flags=w.F32) == -1                # low precision without WL_MIXED
    assert call(flags=w.DAG) == -1
    # a mixed solve needs more scratch than the FP64 one it was sized for
    assert call(flags=w.MIXED) == -2
    assert w.lib.wl_problems_workspace_bytes(arr, 2, w.MIXED) > need
    assert call(tol=-1.0) == -1
    arr[1].dims = w._dims((4, 4, 3, 8))
    assert call() == -1 and "problem 1" in w.last_error()
    assert w.lib.wl_problems_workspace_bytes(arr, 2, 0) == 0
    arr[1].dims = w._dims((4, 4, 4, 8))
    arr[1].x = arr[1].b
    assert call() == -1 and "b == x" in w.last_error()


def test_server_config_checks(w):
    """Every config error is caught before the server touches the device."""
    def cfg(**k):
        c = w.ServerConfig()
        c.hbm_budget = k.get("budget", 1 << 30)
        c.slots = k.get("slots", 4)
        c.flags = k.get("flags", w.EO | w.MIXED)
        c.tol = k.get("tol", 1e-10)
        c.maxiter = k.get("maxiter", 1000)
        c.phases = w._phases(k.get("phases", w.ANTIPERIODIC_T))
        c.merge = k.get("merge", 1)
        c.site_slack = k.get("site_slack", 0.0)
        return c
    h = ctypes.c_void_p()
    create = lambda **k: w.lib.wl_server_create(ctypes.byref(cfg(**k)), ctypes.byref(h))
    assert create(budget=0) == -1 and "budget" in w.last_error()
    assert create(slots=0) == -1 and create(slots=65) == -1
    assert create(merge=-1) == -1 and create(merge=65) == -1 and "merge" in w.last_error()
    assert create(flags=w.F32) == -1                 # low precision without WL_MIXED
    assert create(flags=w.DAG) == -1
    assert create(tol=0.0) == -1
    assert create(maxiter=0) == -1
    assert create(phases=(1, 1, 1, 2)) == -1
    assert create(site_slack=-1e-9) == -1 and "site_slack" in w.last_error()
    assert create(site_slack=float("nan")) == -1 and create(site_slack=float("inf")) == -1
    assert create(flags=w.EO | w.CANON) == -1 and "packed" in w.last_error()
    assert w.lib.wl_server_create(None, ctypes.byref(h)) == -1
    assert h.value is None
    # calls on no server fail cleanly
    t = ctypes.c_uint64()
    assert w.lib.wl_server_submit(None, None, ctypes.byref(t)) == -1
    assert w.lib.wl_server_wait(None, 1, None, None) == -1
    assert w.lib.wl_server_next(None, ctypes.byref(t), None, None) == -1
    assert w.lib.wl_server_pending(None) == 0
    assert w.lib.wl_server_destroy(None) == 0


def test_stream_copy_checks(w):
    lib = w.lib
    assert lib.wl_stream_copy(None, _p(4096), 64, None) == -1
    assert lib.wl_stream_copy(_p(4096), _p(8192), 65, None) == -1       # size not a multiple of 16
    assert lib.wl_stream_copy(_p(4104), _p(8192), 64, None) == -1       # misaligned
    assert lib.wl_stream_copy(_p(4096), _p(4096 + 32), 64, None) == -1  # overlap
    assert "overlap" in w.last_error()


def test_noalloc_solve_rejects_before_touching_the_gpu(w):
    """solve_cg_noalloc refuses, with nothing done, a lattice whose workspace
    exceeds its 64 MiB static scratch, and graph replay (which allocates)."""
    ph = (ctypes.c_double * 8)(1, 0, 1, 0, 1, 0, -1, 0)
    st = w.SolveStats()
    big = w._dims((16, 16, 16, 32))       # FP64 workspace ~ 230 MB
    assert w.workspace_bytes((16, 16, 16, 32), 0) > (64 << 20)
    assert w.lib.solve_cg_noalloc(_p(8), _p(16), _p(32), big, 0.1, ph, 1e-10, 10, 0,
                                  ctypes.byref(st), None) == w.EWORKSPACE
    assert b"static scratch" in w.lib.wl_last_error()
    small = w._dims((4, 4, 4, 4))
    assert w.lib.solve_cg_noalloc(_p(8), _p(16), _p(32), small, 0.1, ph, 1e-10, 10, w.GRAPH,
                                  ctypes.byref(st), None) == w.EINVAL
    assert w.lib.solve_cg_noalloc(_p(8), _p(16), _p(32), w._dims((4, 4, 4, 5)), 0.1, ph,
                                  1e-10, 10, 0, ctypes.byref(st), None) == w.EINVAL
    # the small configurations of the uneven batch fit
    for d in ((4, 4, 4, 4), (8, 8, 8, 8), (8, 8, 8, 16)):
        assert w.workspace_bytes(d, w.EO | w.MIXED) <= (64 << 20)


def test_host_tensors_are_refused_before_any_call(w):
    """The binding refuses host tensors where the ABI takes device buffers
    (checked before the library is called: nothing launches)."""
    import torch
    U = torch.zeros((256, 4, 3, 3), dtype=torch.complex128)
    with pytest.raises(ValueError):
        w.heatbath(U, (4, 4, 4, 4), 1.0)
    with pytest.raises(ValueError):
        w._ptr(torch.zeros(4))


def test_canonical_workspace(w):
    """WL_CANON adds the packed gauge field, b and x (each on a 256-byte
    boundary) after the solver's own workspace; batches do not take it."""
    up = lambda v: (v + 255) // 256 * 256
    for d in ((4, 4, 4, 4), (6, 4, 6, 10)):
        for f in (w.EO, w.EO | w.MIXED, w.EO | w.MIXED | w.F16S | w.LINK12):
            base = w.workspace_bytes(d, f)
            canon = w.workspace_bytes(d, f | w.CANON)
            want = up(up(up(base) + w.gauge_bytes(d, f & w.LINK12)) + w.spinor_bytes(d)) + \
                w.spinor_bytes(d)
            assert canon == want, (d, f)
        assert w.workspace_bytes(d, w.EO | w.CANON, 3) == 0


def test_profiled_traffic_matches_the_kernel_sources():
    """The HBM traffic the benchmark reports comes from committed counter runs
    of the hopping kernels; it is valid only for the sources those runs
    measured, which the profile records by hash. A change to those sources
    must come with new counter runs."""
    import importlib.util
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_for_hash", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    with open(os.path.join(root, "profiles", "hop_f32_eo_32x64_pmc.json")) as f:
        prof = json.load(f)
    assert prof["source_hash"] == bench.kernel_source_hash()
    assert bench.profiled_traffic(False) and bench.profiled_traffic(False, fp64=True)
