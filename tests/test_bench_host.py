"""Host-side logic of bench.py that needs no GPU: the one-GPU contract and
the field rotation that keeps cache-sized operands out of the Infinity
Cache."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_rotated_copies_exceed_the_infinity_cache():
    b = _bench()
    cache = 256 << 20
    # working sets of the cache-sized lattices the benchmark rotates: 16^3x32
    # FP64-18 / FP32-12 and the 32^3x8 local volume in FP64
    for ws in (126 << 20, 40 << 20, 251 << 20, 1, cache, 2 * cache):
        n = b.rotation_copies(ws)
        assert n >= 2
        assert n * ws >= b.ROTATE_BYTES > 2 * cache
        assert n == 2 or (n - 1) * ws < b.ROTATE_BYTES   # no more copies than needed
