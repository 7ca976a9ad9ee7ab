#!/usr/bin/env python3
"""Benchmark of the Wilson-Dirac hot path on one MI355X.

Workload (default): the 32^3 x 64 lattice (2,097,152 sites), links
exp(i eps H) with eps = 0.35 (seed 0), kappa = 0.155, Gaussian source (seed 1),
antiperiodic time. One step = pack the resident source, an even-odd
preconditioned mixed-precision CG solve (FP32 Krylov iterations with FP64
reliable updates) to ||b - M x|| / ||b|| <= 1e-10 recomputed in FP64, and
unpack the solution.

Printed: stdout ends with one compact JSON line (the headline): ``value`` is
the whole-step throughput in algorithmic (compulsory) GB/s -- the library's
per-kernel byte model summed over the step, divided by the step's wall time;
``roofline`` describes the dominant kernel (the FP32 even-odd hopping term)
timed with HIP events on the stream it runs on, ``roofline_fp64_eo`` the
paper's measured kernel (the FP64 even-odd hop); ``cpu_baseline`` times a
bounded run of the FP64 CPU oracle's even-odd CGNR on the same system (all
host threads); ``serving`` summarises the served streams. Everything else
(every Dslash variant, the small configurations, the 12 point sources of a
24^3 x 48 propagator and their meson correlators, the uneven batch of 64
small lattices, the served Poisson streams by size, a twisted-mass solve, the
heat bath, plaquette and an overlapped configuration chain, the autotuner's
record) goes to stderr and, as JSON, to the file ``--detail`` names.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# algorithmic bytes per site of one spinor, and per complex link entry, by
# storage: FP64, FP32, FP16 (24 halves plus one FP32 scale per spinor)
SPINOR_BYTES = {0x0: 192, 0x1: 96, 0x2: 52}
COMPLEX_BYTES = {0x0: 16, 0x1: 8, 0x2: 4}

WORKLOADS = {
    # name: dims, kappa, eps
    "32^3x64": ((32, 32, 32, 64), 0.155, 0.35),
    "16^3x32": ((16, 16, 16, 32), 0.15, 0.30),
    "8^3x16": ((8, 8, 8, 16), 0.15, 0.30),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="32^3x64", choices=sorted(WORKLOADS))
    ap.add_argument("--link12", action="store_true", help="12-real link storage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--kernel-launches", type=int, default=50)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 12-point-source and 64-lattice batch measurements")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 4^4 and 16^3x32 configurations")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-budget-gb", type=float, default=64.0)
    ap.add_argument("--detail", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file (relative to this script's folder) for the full results")
    ap.add_argument("--serving-merge", type=int, default=8,
                    help="most waiting requests of one size served as one batch")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the sources that define the hopping kernels (their code, layout and reductions)
HOP_SOURCES = ("wl_hop.h", "wl_hop_f32.hip", "wl_hop_f64.hip", "wl_dslash.hip", "wl_internal.h",
               "wl_reduce.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1112_5280_amd", "csrc")
    for f in HOP_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(link12, fp64=False):
    """Bytes per launch of the FP32 (or, with fp64, the FP64) even-odd hop from
    the committed PMC summary (FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy's readings), or None when the summary is for another kernel or the
    kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "hop_f32_eo_32x64_pmc.json")
    if link12 or not os.path.exists(path):
        return None
    with open(path) as f:
        pm = json.load(f)
    if pm.get("source_hash") != kernel_source_hash():
        return None
    if fp64:
        return pm.get("fp64_eo_hop", {}).get("traffic_bytes_per_launch")
    return pm["traffic_bytes_per_launch"]


def time_kernel(fn, n, torch):
    """Average duration of one launch of fn(), in seconds: a pair of HIP events
    around each of n launches on the launch stream (gaps between launches are
    not counted, as in a profiler's per-dispatch durations)."""
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    for e0, e1 in ev:
        e0.record(s)
        fn()
        e1.record(s)
    ev[-1][1].synchronize()
    return sum(e0.elapsed_time(e1) for e0, e1 in ev) / 1e3 / n


def time_kernel_rot(fns, n, torch):
    """time_kernel over launches that take fns[0], fns[1], ... in turn: each
    callable works on its own copy of the fields, and the copies together are
    larger than the 256 MB Infinity Cache, so a launch finds its operands in
    HBM rather than left in the cache by the launch before it."""
    k = [0]

    def step():
        fns[k[0] % len(fns)]()
        k[0] += 1

    for f in fns:
        f()
    return time_kernel(step, n, torch)


# total size of the field copies rotated through when an operator's working
# set would otherwise stay in the 256 MB Infinity Cache
ROTATE_BYTES = 600 << 20


def rotation_copies(ws_bytes):
    return max(2, -(-ROTATE_BYTES // ws_bytes))


def timed(fn, torch):
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


def batch12(w, torch, synth, n_launch):
    """The 12 spin-colour point sources on the 24^3 x 48 lattice (eps = 0.3,
    kappa = 0.15): batched M GB/s at 432 B per site-RHS (FP64-18), and the
    batched eo-CG solves of all 12 (FP64, graph replay, FP32 and FP16 inner)
    against 12 solo solves."""
    dims, kappa = (24, 24, 24, 48), 0.15
    V = synth.volume(dims)
    U = synth.gauge_smooth(dims, 0.30, 0)
    site = synth.random_site(dims, 2)
    n = 12
    out = {"lattice": list(dims), "kappa": kappa, "source_site": site}
    s = torch.cuda.current_stream()
    ops = {}
    for prec, lk, name in ((w.F64, w.LINK18, "f64_18"), (w.F32, w.LINK18, "f32_18"),
                           (w.F32, w.LINK12, "f32_12")):
        G = w.pack_gauge(U, dims, prec | lk)
        B = w.empty_batch(dims, n, prec)
        for r in range(n):
            w.batch_field(B, dims, prec, r).copy_(
                w.pack_spinor(synth.point_source(dims, site, r // 3, r % 3), dims, prec))
        O = w.empty_batch(dims, n, prec)
        f = prec | lk
        tm = time_kernel(lambda: w.wilson_dslash_batch(G, B, O, n, dims, kappa, flags=f,
                                                       stream=s), n_launch, torch)
        per = 2 * SPINOR_BYTES[prec] + 4 * COMPLEX_BYTES[prec] * (6 if lk else 9) / n
        P1 = w.batch_field(B, dims, prec, 0)
        O1 = w.empty_spinor(dims, prec)
        t1 = time_kernel(lambda: w.wilson_dslash(G, P1, O1, dims, kappa, flags=f, stream=s),
                         n_launch, torch)
        ops["M_batch12_" + name] = {
            "us": tm * 1e6, "bytes_per_site_rhs": per, "GBs": per * V * n / tm / 1e9,
            "GFLOPs": 1368.0 * V * n / tm / 1e9, "single_rhs_us": t1 * 1e6,
            "speedup_vs_12_single": 12 * t1 / tm}
        del G, B, O, O1
    out["dslash"] = ops
    torch.cuda.empty_cache()

    G = w.pack_gauge(U, dims, w.F64)
    B = w.empty_batch(dims, n)
    for r in range(n):
        w.batch_field(B, dims, 0, r).copy_(
            w.pack_spinor(synth.point_source(dims, site, r // 3, r % 3), dims))
    X = w.empty_batch(dims, n)
    solves = {}
    for f, name in ((w.EO, "batched_f64_eo"), (w.EO | w.GRAPH, "batched_f64_eo_graph"),
                    (w.EO | w.MIXED, "batched_mixed_f32_eo"),
                    (w.EO | w.MIXED | w.F16S, "batched_mixed_f16_eo")):
        work = torch.empty(w.workspace_bytes(dims, f, n), dtype=torch.uint8, device="cuda")
        # warm-up: the first call tunes the batched launch shapes
        w.solve_cg_batch(G, B, X, n, dims, kappa, flags=f, work=work, stream=s)
        (code, st), dt = timed(lambda: w.solve_cg_batch(G, B, X, n, dims, kappa, flags=f,
                                                        work=work, stream=s), torch)
        assert code == 0 and max(x["true_res"] for x in st) <= 1e-10, st
        solves[name] = {"seconds": dt, "solves_per_s": n / dt,
                        "iterations_max": max(x["iterations"] for x in st),
                        "true_res_max": max(x["true_res"] for x in st)}
        del work
    # the meson correlators of Eq. 1 from the 12 propagator columns just solved
    t0 = site // (dims[0] * dims[1] * dims[2])
    mw = torch.empty(w.lib.wl_meson_workspace_bytes(w._dims(dims)), dtype=torch.uint8,
                     device="cuda")
    tmes = time_kernel(lambda: w.meson_correlators(X, dims, t0, work=mw, stream=s), n_launch,
                       torch)
    corr = w.meson_correlators(X, dims, t0, work=mw, stream=s).cpu()
    out["meson_correlators"] = {
        "us": tmes * 1e6, "GBs": 12 * V * 192 / tmes / 1e9,
        "pion_C15": [float(v) for v in corr[15].real[:6]],
        "note": "C_Gamma(t) of Eq. 1 for the 16 Gamma_n, t from the source slice; "
                "GB/s counts the 12 FP64 propagator columns read once"}
    del mw
    X1 = w.empty_spinor(dims)
    for f, name in ((w.EO, "sequential_f64_eo"), (w.EO | w.MIXED, "sequential_mixed_f32_eo"),
                    (w.EO | w.MIXED | w.F16S, "sequential_mixed_f16_eo")):
        work = torch.empty(w.workspace_bytes(dims, f), dtype=torch.uint8, device="cuda")
        def run():
            return [w.solve_cg(G, w.batch_field(B, dims, 0, r), X1, dims, kappa, flags=f,
                               work=work, stream=s) for r in range(n)]
        w.solve_cg(G, w.batch_field(B, dims, 0, 0), X1, dims, kappa, flags=f, work=work,
                   stream=s)
        st, dt = timed(run, torch)
        assert all(x["status"] == 0 and x["true_res"] <= 1e-10 for x in st), st
        solves[name] = {"seconds": dt, "solves_per_s": n / dt,
                        "iterations_max": max(x["iterations"] for x in st),
                        "true_res_max": max(x["true_res"] for x in st)}
        del work
    out["solves"] = solves
    out["batched_vs_sequential_f64"] = (solves["sequential_f64_eo"]["seconds"] /
                                        solves["batched_f64_eo"]["seconds"])
    out["batched_vs_sequential_mixed_f32"] = (solves["sequential_mixed_f32_eo"]["seconds"] /
                                              solves["batched_mixed_f32_eo"]["seconds"])
    out["autotuned_rhs_per_thread"] = w.tuning_report().strip().splitlines()
    del G, B, X, X1
    torch.cuda.empty_cache()
    return out


def pure_gauge(w, torch, synth, np, U_host, dims, n_launch):
    """The heat bath and the plaquette on the bench lattice (canonical and
    packed fields), and the chain of
    configurations with overlapped measurement (paper Sec. 3 and Sec. 4):
    heat-bath sweep time, link updates per second, plaquette kernel time, and
    the seconds per configuration of a 16^3 x 32 chain (2 sweeps per
    configuration; its 12 point-source propagator solves and meson
    correlators) with and without the two-stream overlap, whose correlators
    must agree bitwise."""
    from paper_1112_5280_amd.ensemble import Ensemble
    V = int(np.prod(dims))
    U = torch.from_numpy(U_host).to("cuda")     # the bench field, heat-bathed in place
    s = torch.cuda.current_stream()
    sweep = [0]

    def one_sweep():
        w.heatbath(U, dims, 5.7, nsweeps=1, sweep0=sweep[0], seed=11, stream=s)
        sweep[0] += 1
    th = time_kernel(one_sweep, max(2, n_launch // 10), torch)
    out = {"lattice": list(dims), "beta": 5.7,
           "heatbath_ms_per_sweep": th * 1e3,
           "link_updates_per_s": 4 * V / th,
           "heatbath_note": "one sweep = 8 launches (4 directions x 2 parities), each link "
                            "3 SU(2) subgroup draws (Kennedy-Pendleton for alpha >= 1, unit-disk "
                            "rejection below) from its 6 staples"}
    out_d = torch.empty(1, dtype=torch.float64, device="cuda")
    pw = torch.empty(max(int(w.lib.wl_plaquette_workspace_bytes(w._dims(dims))), 8),
                     dtype=torch.uint8, device="cuda")
    tp = time_kernel(lambda: w.lib.wl_plaquette(w._ptr(U), w._dims(dims), w._ptr(out_d),
                                                w._ptr(pw), pw.numel(), w._stream(s)),
                     n_launch, torch)
    out.update({"plaquette": w.plaquette(U, dims), "plaquette_us": tp * 1e6,
                "plaquette_GBs": 4 * V * 144 / tp / 1e9})
    # the same two on the packed FP64 field (coalesced loads; the heat bath is
    # bitwise the canonical one)
    G = w.pack_gauge(U, dims)

    def one_sweep_packed():
        w.heatbath_packed(G, dims, 5.7, nsweeps=1, sweep0=sweep[0], seed=11, stream=s)
        sweep[0] += 1
    thp = time_kernel(one_sweep_packed, max(2, n_launch // 10), torch)
    tpp = time_kernel(lambda: w.lib.wl_plaquette_packed(w._ptr(G), w._dims(dims), w._ptr(out_d),
                                                        w._ptr(pw), pw.numel(), w._stream(s)),
                      n_launch, torch)
    out.update({"heatbath_packed_ms_per_sweep": thp * 1e3,
                "link_updates_per_s_packed": 4 * V / thp,
                "plaquette_packed_us": tpp * 1e6,
                "plaquette_packed_GBs": 4 * V * 144 / tpp / 1e9})
    del U, G, pw
    torch.cuda.empty_cache()
    d2 = (16, 16, 16, 32)
    U0 = synth.gauge_unit(d2)
    chain = {}
    for ov in (True, False):
        e = Ensemble(U0, d2, 5.7, sweeps=2, kappa=0.12, site=0, seed=3, overlap=ov)
        e.run(1)                                    # warm-up: tuning, graphs
        torch.cuda.synchronize()
        t = time.perf_counter()
        corr = e.run(4)
        chain[ov] = (corr, (time.perf_counter() - t) / 4, e.stats[-1])
        del e
    assert torch.equal(chain[True][0], chain[False][0])
    out["chain_16x16x16x32"] = {
        "seconds_per_configuration_overlapped": chain[True][1],
        "seconds_per_configuration_sequential": chain[False][1],
        "iterations": max(x["iterations"] for x in chain[True][2]),
        "correlators_bitwise_equal": True}
    torch.cuda.empty_cache()
    return out


def uneven64(w, torch, synth, np):
    """64 independent lattices, sizes uniform over {4^4, 8^4, 8^3 x 16}, kappa
    uniform in [0.10, 0.14] (seed 3), Haar gauge fields and Gaussian sources of
    their own seeds: one solve_cg_problems call against 64 solo solves."""
    sizes = ((4, 4, 4, 4), (8, 8, 8, 8), (8, 8, 8, 16))
    rng = np.random.default_rng(3)
    probs = []
    for i in range(64):
        dims = sizes[rng.integers(3)]
        kappa = float(rng.uniform(0.10, 0.14))
        G = w.pack_gauge(synth.gauge_haar(dims, 100 + i), dims)
        B = w.pack_spinor(synth.gaussian_spinor(dims, 200 + i), dims)
        probs.append(w.Problem(dims, kappa, G, B, w.zeros_spinor(dims)))
    s = torch.cuda.current_stream()
    out = {"lattices": 64, "sites_total": int(sum(synth.volume(p.dims) for p in probs))}
    for f, name in ((w.EO, "f64_eo"), (w.EO | w.GRAPH, "f64_eo_graph"),
                    (w.EO | w.MIXED, "mixed_f32_eo")):
        work = torch.empty(w.problems_workspace_bytes(probs, f), dtype=torch.uint8,
                           device="cuda")
        w.solve_cg_problems(probs, flags=f, work=work, stream=s)      # warm-up
        (code, st), dt = timed(lambda: w.solve_cg_problems(probs, flags=f, work=work,
                                                           stream=s), torch)
        assert code == 0 and max(x["true_res"] for x in st) <= 1e-10
        out["batched_" + name] = {"seconds": dt, "lattice_solves_per_s": 64 / dt,
                                  "iterations_max": max(x["iterations"] for x in st),
                                  "algorithmic_GBs": sum(x["bytes"] for x in st) / dt / 1e9}
        wk = {}
        for p in probs:
            if p.dims not in wk:
                wk[p.dims] = torch.empty(w.workspace_bytes(p.dims, f), dtype=torch.uint8,
                                         device="cuda")
        def run():
            return [w.solve_cg(p.gauge, p.b, p.x, p.dims, p.kappa, flags=f, work=wk[p.dims],
                               stream=s) for p in probs]
        run()
        st, dt = timed(run, torch)
        assert all(x["status"] == 0 for x in st)
        out["sequential_" + name] = {"seconds": dt, "lattice_solves_per_s": 64 / dt}
        del work, wk
    out["batched_vs_sequential"] = (out["sequential_f64_eo"]["seconds"] /
                                    out["batched_f64_eo"]["seconds"])
    out["batched_graph_vs_sequential"] = (out["sequential_f64_eo"]["seconds"] /
                                          out["batched_f64_eo_graph"]["seconds"])
    return out


def small_configs(w, torch, synth, n_launch):
    """The two small configurations. 4^4 (Haar, kappa 0.12, FP64): one M apply
    and a CGNR solve -- latency-bound, reported in microseconds. 16^3 x 32
    (exp(i 0.3 H), kappa 0.15): every operator variant (its working set fits in
    the 256 MB Infinity Cache, so these rates are cache-resident, not HBM; each
    is timed again over rotated copies of its fields, from HBM) and BiCGStab on
    the even-odd system, plain FP64 and mixed."""
    s = torch.cuda.current_stream()
    out = {}
    dims, kappa = (4, 4, 4, 4), 0.12
    U = synth.gauge_haar(dims, 0)
    b = synth.gaussian_spinor(dims, 1)
    G = w.pack_gauge(U, dims)
    B = w.pack_spinor(b, dims)
    O = w.empty_spinor(dims)
    t = time_kernel(lambda: w.wilson_dslash(G, B, O, dims, kappa, stream=s), n_launch, torch)
    c1 = {"lattice": list(dims), "M_apply_us": t * 1e6}
    X = w.empty_spinor(dims)
    for f, name in ((0, "cg_full_f64"), (w.EO, "cg_eo_f64"), (w.EO | w.GRAPH, "cg_eo_f64_graph")):
        w.solve_cg(G, B, X, dims, kappa, flags=f, stream=s)
        st, dt = timed(lambda: w.solve_cg(G, B, X, dims, kappa, flags=f, stream=s), torch)
        assert st["status"] == 0 and st["true_res"] <= 1e-10, st
        c1[name] = {"us": dt * 1e6, "iterations": st["iterations"], "true_res": st["true_res"]}
    out["4^4"] = c1

    dims, kappa = (16, 16, 16, 32), 0.15
    V = synth.volume(dims)
    U = synth.gauge_smooth(dims, 0.30, 0)
    b = synth.gaussian_spinor(dims, 1)
    ops, hbm = {}, {}
    for prec, pname in ((w.F64, "f64"), (w.F32, "f32")):
        for lk, lname in ((w.LINK18, "18"), (w.LINK12, "12")):
            G = w.pack_gauge(U, dims, prec | lk)
            P = w.pack_spinor(b, dims, prec)
            O = w.empty_spinor(dims, prec)
            Oh = w.empty_spinor(dims, prec, 1)
            per = 2 * SPINOR_BYTES[prec] + 4 * COMPLEX_BYTES[prec] * (6 if lk else 9)
            for dag, dname in ((0, "M"), (w.DAG, "Mdag")):
                f = prec | lk | dag
                tm = time_kernel(lambda: w.wilson_dslash(G, P, O, dims, kappa, flags=f, stream=s),
                                 n_launch, torch)
                ops["%s_%s_%s" % (dname, pname, lname)] = {
                    "us": tm * 1e6, "GBs": per * V / tm / 1e9, "GFLOPs": 1368 * V / tm / 1e9}
            f = prec | lk | w.HOP
            te = time_kernel(lambda: w.wilson_dslash_eo(G, w.parity_block(P, dims, prec, 0), Oh,
                                                        dims, kappa, 1, flags=f, stream=s),
                             n_launch, torch)
            ops["Deo_%s_%s" % (pname, lname)] = {
                "us": te * 1e6, "GBs": (per + 4 * COMPLEX_BYTES[prec] * (6 if lk else 9)) * V / 2 / te / 1e9,
                "GFLOPs": 1320 * V / 2 / te / 1e9}
            # the same launches with their operands in HBM: copies of the fields
            # rotated so that no launch finds them in the Infinity Cache
            ws = G.numel() + P.numel() + O.numel() + Oh.numel()
            nc = rotation_copies(ws)
            cp = [(G, P, O, Oh)] + [(G.clone(), P.clone(), torch.empty_like(O),
                                     torch.empty_like(Oh)) for _ in range(nc - 1)]
            tm = time_kernel_rot([lambda c=c: w.wilson_dslash(c[0], c[1], c[2], dims, kappa,
                                                              flags=prec | lk, stream=s)
                                  for c in cp], n_launch, torch)
            te = time_kernel_rot([lambda c=c: w.wilson_dslash_eo(
                c[0], w.parity_block(c[1], dims, prec, 0), c[3], dims, kappa, 1,
                flags=prec | lk | w.HOP, stream=s) for c in cp], n_launch, torch)
            hbm["M_%s_%s" % (pname, lname)] = {"us": tm * 1e6, "GBs": per * V / tm / 1e9,
                                               "copies": nc}
            hbm["Deo_%s_%s" % (pname, lname)] = {
                "us": te * 1e6,
                "GBs": (per + 4 * COMPLEX_BYTES[prec] * (6 if lk else 9)) * V / 2 / te / 1e9,
                "copies": nc}
            del cp
    G = w.pack_gauge(U, dims)
    B = w.pack_spinor(b, dims)
    X = w.empty_spinor(dims)
    solves = {}
    for f, name in ((w.EO, "bicgstab_eo_f64"), (w.EO | w.MIXED, "bicgstab_eo_mixed_f32"),
                    (w.EO | w.MIXED | w.F16S, "bicgstab_eo_mixed_f16"), (w.EO, "cg_eo_f64"),
                    (w.EO | w.MIXED, "cg_eo_mixed_f32")):
        fn = w.solve_bicgstab if name.startswith("bicgstab") else w.solve_cg
        st, dt = timed(lambda: fn(G, B, X, dims, kappa, maxiter=60000, flags=f, stream=s), torch)
        solves[name] = {"ms": dt * 1e3, "status": st["status_name"], "iterations": st["iterations"],
                        "fp64_iterations": st["fp64_iterations"], "restarts": st["restarts"],
                        "true_res": st["true_res"]}
    out["16^3x32"] = {"lattice": list(dims), "kappa": kappa, "cache_resident": True,
                      "operators": ops, "operators_hbm": hbm, "solves": solves}

    # one GPU's share of 32^3x64 cut into 8 along t: the 32^3x8 local volume
    # (periodic here; over 8 GPUs its two t faces, one spin-projected half
    # spinor of 6 complex per face site each, come from the neighbours)
    dims, kappa = (32, 32, 32, 8), 0.155
    V = synth.volume(dims)
    U = synth.gauge_smooth(dims, 0.35, 0)
    b = synth.gaussian_spinor(dims, 1)
    face = dims[0] * dims[1] * dims[2]
    loc = {"lattice": list(dims), "face_sites": face}
    for prec, pname in ((w.F64, "f64"), (w.F32, "f32")):
        G = w.pack_gauge(U, dims, prec)
        P = w.pack_spinor(b, dims, prec)
        O = w.empty_spinor(dims, prec)
        Oh = w.empty_spinor(dims, prec, 1)
        lb = 9 * COMPLEX_BYTES[prec]
        tm = time_kernel(lambda: w.wilson_dslash(G, P, O, dims, kappa, flags=prec, stream=s),
                         n_launch, torch)
        te = time_kernel(lambda: w.wilson_dslash_eo(G, w.parity_block(P, dims, prec, 0), Oh,
                                                    dims, kappa, 1, flags=prec | w.HOP,
                                                    stream=s), n_launch, torch)
        loc["M_%s_18" % pname] = {"us": tm * 1e6,
                                  "GBs": (2 * SPINOR_BYTES[prec] + 4 * lb) * V / tm / 1e9}
        loc["Deo_%s_18" % pname] = {"us": te * 1e6,
                                    "GBs": (2 * SPINOR_BYTES[prec] + 8 * lb) * V / 2 / te / 1e9}
        # a local volume's fields fit in the Infinity Cache (FP64: 251 MB); the
        # same launches over rotated copies give the HBM rate
        ws = G.numel() + P.numel() + O.numel() + Oh.numel()
        nc = rotation_copies(ws)
        cp = [(G, P, O, Oh)] + [(G.clone(), P.clone(), torch.empty_like(O), torch.empty_like(Oh))
                                for _ in range(nc - 1)]
        tm = time_kernel_rot([lambda c=c: w.wilson_dslash(c[0], c[1], c[2], dims, kappa,
                                                          flags=prec, stream=s)
                              for c in cp], n_launch, torch)
        te = time_kernel_rot([lambda c=c: w.wilson_dslash_eo(
            c[0], w.parity_block(c[1], dims, prec, 0), c[3], dims, kappa, 1,
            flags=prec | w.HOP, stream=s) for c in cp], n_launch, torch)
        loc["M_%s_18_hbm" % pname] = {"us": tm * 1e6, "copies": nc,
                                      "GBs": (2 * SPINOR_BYTES[prec] + 4 * lb) * V / tm / 1e9}
        loc["Deo_%s_18_hbm" % pname] = {
            "us": te * 1e6, "copies": nc,
            "GBs": (2 * SPINOR_BYTES[prec] + 8 * lb) * V / 2 / te / 1e9}
        loc["face_bytes_%s" % pname] = 6 * COMPLEX_BYTES[prec] * face
        del G, P, O, Oh, cp
    out["32^3x8_local_volume"] = loc
    return out


SERVE_SIZES = (((8, 8, 8, 8), 0.40), ((16, 16, 16, 32), 0.35), ((24, 24, 24, 48), 0.20),
               ((32, 32, 32, 64), 0.05))


# the earliest-deadline admission's slack per lattice site: a 32^3x64 request
# (2.1M sites) may be overtaken by smaller ones for up to 0.42 s, a 24^3x48 one
# for 0.13 s. Measured at 0.5 / 0.8 of saturation against 2e-8 and 5e-8 (and
# first in first out): the lowest p99 at 0.5 S and the lowest p50 at 0.8 S.
SERVE_SLACK = 2e-7


def serving(w, torch, synth, np, n_req, budget_gb, slots, merge, slacks=(SERVE_SLACK,)):
    """Poisson stream of solve requests against 8 resident gauge fields (two
    exp(i 0.3 H) fields per lattice size, seeds 0..7): sizes 8^4 40 %, 16^3x32
    35 %, 24^3x48 20 %, 32^3x64 5 %; kappa uniform in [0.12, 0.155]; Gaussian
    sources (two per size, drawn once); arrivals, sizes, kappas and choices
    from seed 4. First the closed-loop saturation rate S (every request queued
    at once), then open-loop streams at 0.5 S and 0.8 S through the server
    (mixed precision, FP16-storage inner solve, `slots` concurrent solves,
    up to `merge` waiting requests of one size solved as one batch, HBM budget
    for workspaces; first in first out, then earliest deadline first with
    `slacks` seconds per lattice site), then the 0.5 S stream through a
    one-slot plain-FP64 server without merging. Latency = arrival to
    solution ready."""
    import queue
    import threading
    t = time.time()
    fields, sources, xpool = {}, {}, {}
    npool = {0: 128, 1: 64, 2: 24, 3: 12}
    for k, (dims, _) in enumerate(SERVE_SIZES):
        fields[k] = [w.pack_gauge(synth.gauge_smooth(dims, 0.30, 2 * k + j), dims)
                     for j in range(2)]
        sources[k] = [w.pack_spinor(synth.gaussian_spinor(dims, 100 + 2 * k + j), dims)
                      for j in range(2)]
        xpool[k] = queue.Queue()
        for _ in range(npool[k]):
            xpool[k].put(w.zeros_spinor(dims))
    log("serving inputs generated in %.1f s" % (time.time() - t))
    probs = np.array([p for _, p in SERVE_SIZES])

    def draw(n, seed):
        rng = np.random.default_rng(seed)
        size = rng.choice(len(SERVE_SIZES), size=n, p=probs)
        kappa = rng.uniform(0.12, 0.155, size=n)
        fld = rng.integers(0, 2, size=n)
        src = rng.integers(0, 2, size=n)
        gaps = rng.exponential(1.0, size=n)   # unit-rate inter-arrival gaps
        return size, kappa, fld, src, gaps

    def run(flags, nslots, rate, n, seed, warm, nmerge, slack=0.0):
        """One stream; rate None = closed loop (all queued at t = 0)."""
        size, kappa, fld, src, gaps = draw(n + warm, seed)
        arrive = np.zeros(n + warm) if rate is None else np.cumsum(gaps) / rate
        lat, lag, status, iters = [], [], [], []
        lat_k = {k: [] for k in range(len(SERVE_SIZES))}
        done_t = []
        srv = w.Server(hbm_budget=int(budget_gb * (1 << 30)), slots=nslots, flags=flags,
                       maxiter=20000, merge=nmerge, site_slack=slack)
        held = {}
        stalls = [0]

        submitted = threading.Semaphore(0)
        errors = []

        def collector():
            try:
                for j in range(n + warm):
                    submitted.acquire()          # next() needs an uncollected request
                    ticket, code, st, tm = srv.next()
                    i, k, x, late = held.pop(ticket)
                    xpool[k].put(x)
                    if i >= warm:
                        lat.append(tm["finished"] - tm["submitted"] + late)
                        lat_k[k].append(lat[-1])
                        status.append(st["status"])
                        iters.append(st["iterations"])
                        done_t.append(tm["finished"])
                    if (j + 1) % 250 == 0:
                        log("  %d of %d requests done" % (j + 1, n + warm))
            except Exception as e:               # surfaced by the submitting thread
                errors.append(e)

        th = threading.Thread(target=collector, daemon=True)
        th.start()
        t0 = time.perf_counter()
        first = None
        for i in range(n + warm):
            dt = arrive[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            k = int(size[i])
            try:
                x = xpool[k].get_nowait()
            except queue.Empty:
                stalls[0] += 1
                while True:
                    if errors:
                        raise errors[0]
                    try:
                        x = xpool[k].get(timeout=1.0)
                        break
                    except queue.Empty:
                        pass
            dims = SERVE_SIZES[k][0]
            late = max(0.0, (time.perf_counter() - t0) - arrive[i])
            p = w.Problem(dims, float(kappa[i]), fields[k][int(fld[i])], sources[k][int(src[i])], x)
            held[i + 1] = (i, k, x, late)        # a new server numbers its tickets 1, 2, ...
            tk = srv.submit(p)
            assert tk == i + 1
            submitted.release()
            if i == warm:
                first = time.perf_counter()
        while th.is_alive():
            th.join(timeout=1.0)
            if errors:
                raise errors[0]
        if errors:
            raise errors[0]
        span = time.perf_counter() - first
        srv.close()
        lat = np.array(lat) * 1e3
        ok = int(sum(1 for s in status if s == 0))
        return {"requests": n, "warmup_requests": warm, "slots": nslots, "merge": nmerge,
                "site_slack": slack, "offered_rate": rate, "solves_per_s": n / span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                "converged": ok, "mean_iterations": float(np.mean(iters)),
                "buffer_stalls": stalls[0],
                "by_size": {"x".join(map(str, SERVE_SIZES[k][0])): {
                    "requests": len(v), "p50_ms": float(np.percentile(v, 50)) * 1e3,
                    "p99_ms": float(np.percentile(v, 99)) * 1e3} for k, v in lat_k.items() if v}}

    mixed = w.EO | w.MIXED | w.F16S
    out = {"hbm_budget_gb": budget_gb, "sizes": [[list(d), p] for d, p in SERVE_SIZES],
           "kappa": [0.12, 0.155], "resident_fields": 8,
           "solver": "eo CG, FP16-storage inner, FP64 reliable updates, tol 1e-10",
           "fp64_solver": "eo CG in FP64, one request at a time, tol 1e-10"}
    # closed-loop saturation of each server (every request queued at once),
    # each on exactly the requests of its 0.8 S stream (same count, warm-up
    # and seed): the requests span 1 ms to a quarter second, so a smaller or
    # other sample misjudges that stream's capacity and the "0.8" load can
    # exceed it
    sat = run(mixed, slots, None, n_req, 41, 20, merge)
    S = sat["solves_per_s"]
    out["closed_loop"] = sat
    out["saturation_solves_per_s"] = S
    n64 = max(100, n_req // 2)
    sat64 = run(w.EO, 1, None, n64, 41, 10, 1)
    S64 = sat64["solves_per_s"]
    out["fp64_closed_loop"] = sat64
    out["fp64_saturation_solves_per_s"] = S64
    log("serving: closed-loop saturation %.1f solves/s (mixed, %d slots), %.1f (FP64, 1 slot)"
        % (S, slots, S64))
    # each server at 0.5 and 0.8 of its own saturation
    for frac, seed in ((0.5, 4), (0.8, 41)):
        r = run(mixed, slots, frac * S, n_req, seed, 20, merge)
        out["open_loop_%.1fS" % frac] = r
        log("serving: mixed at %.1f S: %.1f solves/s, p50 %.1f ms, p99 %.1f ms"
            % (frac, r["solves_per_s"], r["p50_ms"], r["p99_ms"]))
    # the same streams, admitted earliest deadline first
    for sl in slacks:
        for frac, seed in ((0.5, 4), (0.8, 41)):
            r = run(mixed, slots, frac * S, n_req, seed, 20, merge, sl)
            key = "open_loop_%.1fS_edf" % frac
            out[key if len(slacks) == 1 else "%s_%g" % (key, sl)] = r
            log("serving: mixed at %.1f S, deadlines %g s/site: %.1f solves/s, p50 %.1f ms, "
                "p99 %.1f ms" % (frac, sl, r["solves_per_s"], r["p50_ms"], r["p99_ms"]))
    for frac, seed in ((0.5, 4), (0.8, 41)):
        r = run(w.EO, 1, frac * S64, n64, seed, 10, 1)
        out["fp64_open_loop_%.1fS64" % frac] = r
        log("serving: FP64 at %.1f S64: %.1f solves/s, p50 %.1f ms, p99 %.1f ms"
            % (frac, r["solves_per_s"], r["p50_ms"], r["p99_ms"]))
    # the mixed server on the very stream the FP64 server got at 0.5 S64: one
    # offered rate below both capacities, so both latencies are service times
    r = run(mixed, slots, 0.5 * S64, n64, 4, 10, merge)
    out["mixed_at_0.5S64"] = r
    log("serving: mixed at 0.5 S64: %.1f solves/s, p50 %.1f ms, p99 %.1f ms"
        % (r["solves_per_s"], r["p50_ms"], r["p99_ms"]))
    del fields, sources, xpool
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_1112_5280_amd import synth
    from paper_1112_5280_amd import wilson as w

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dims, kappa, eps = WORKLOADS[args.workload]
    V = synth.volume(dims)
    Vh = V // 2
    link = w.LINK12 if args.link12 else w.LINK18
    t = time.time()
    U = synth.gauge_smooth(dims, eps, 0)
    b = synth.gaussian_spinor(dims, 1)
    log("inputs generated in %.1f s" % (time.time() - t))

    G64 = w.pack_gauge(U, dims, w.F64 | link)
    b_dev = torch.from_numpy(b).to("cuda")
    B = w.empty_spinor(dims)
    X = w.empty_spinor(dims)
    x_dev = torch.empty_like(b_dev)
    flags = w.EO | w.MIXED | link
    work = torch.empty(w.workspace_bytes(dims, flags), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    sp = w._stream(s)
    d4 = w._dims(dims)

    def step():
        w._check(w.lib.wl_pack_spinor(w._ptr(b_dev), w._ptr(B), d4, w.F64, sp), "pack")
        st = w.solve_cg(G64, B, X, dims, kappa, tol=1e-10, maxiter=20000, flags=flags,
                        work=work, stream=s)
        w._check(w.lib.wl_unpack_spinor(w._ptr(X), w._ptr(x_dev), d4, w.F64, sp), "unpack")
        return st

    for _ in range(args.warmup):
        st = step()
        log("warmup solve: status %s, %d iterations, %d outer, true residual %.2e, %.3f s"
            % (st["status_name"], st["iterations"], st["restarts"], st["true_res"],
               st["seconds"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    for st in stats:
        assert st["status"] == 0 and st["true_res"] <= 1e-10, st
    pack_bytes = 2 * V * (192 + 192)           # canonical <-> packed, both ways
    step_bytes = float(np.mean([st["bytes"] for st in stats])) + pack_bytes
    step_flops = float(np.mean([st["flops"] for st in stats]))
    value = step_bytes / (ms / 1e3) / 1e9

    # FP64 solve of the same system on the same GPU, for the mixed-vs-FP64 comparison
    fp64 = None
    if not args.no_fp64_compare:
        X64 = w.empty_spinor(dims)
        w64 = torch.empty(w.workspace_bytes(dims, w.EO | link), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        st64 = w.solve_cg(G64, B, X64, dims, kappa, tol=1e-10, maxiter=20000,
                          flags=w.EO | link, work=w64, stream=s)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        x64 = w.unpack_spinor(X64, dims)
        diff = float(torch.linalg.vector_norm(x64 - x_dev) / torch.linalg.vector_norm(x64))
        fp64 = {"seconds": dt, "iterations": st64["iterations"], "status": st64["status_name"],
                "true_res": st64["true_res"], "mixed_speedup": dt / (ms / 1e3),
                "mixed_vs_fp64_solution_rel_diff": diff}
        del X64, w64, x64

    # the same solve with FP16-storage (per-site scaled) inner iterations
    f16 = None
    if not args.no_fp64_compare:
        f16f = w.EO | w.MIXED | w.F16S | link
        wk = torch.empty(w.workspace_bytes(dims, f16f), dtype=torch.uint8, device="cuda")
        X16 = w.empty_spinor(dims)
        w.solve_cg(G64, B, X16, dims, kappa, tol=1e-10, maxiter=20000, flags=f16f, work=wk,
                   stream=s)
        st16, dt = timed(lambda: w.solve_cg(G64, B, X16, dims, kappa, tol=1e-10,
                                            maxiter=20000, flags=f16f, work=wk, stream=s),
                         torch)
        x16 = w.unpack_spinor(X16, dims)
        f16 = {"seconds": dt, "iterations": st16["iterations"], "status": st16["status_name"],
               "outer_corrections": st16["restarts"], "true_res": st16["true_res"],
               "vs_fp32_inner": (ms / 1e3) / dt,
               "solution_rel_diff_vs_fp32_inner": float(
                   torch.linalg.vector_norm(x16 - x_dev) / torch.linalg.vector_norm(x_dev))}
        del wk, X16, x16

    # the two mixed solves with 12-real link storage (third row rebuilt in the
    # kernels): fewer bytes per hop, so a shorter time to solution
    link12_solves = None
    if not args.no_fp64_compare and not args.link12:
        G12 = w.pack_gauge(U, dims, w.F64 | w.LINK12)
        X12 = w.empty_spinor(dims)
        link12_solves = {}
        for f, name, ref in ((w.EO | w.MIXED | w.LINK12, "mixed_f32", ms / 1e3),
                             (w.EO | w.MIXED | w.F16S | w.LINK12, "mixed_f16",
                              f16["seconds"] if f16 else None)):
            wk = torch.empty(w.workspace_bytes(dims, f), dtype=torch.uint8, device="cuda")
            w.solve_cg(G12, B, X12, dims, kappa, tol=1e-10, maxiter=20000, flags=f, work=wk,
                       stream=s)
            st12, dt = timed(lambda: w.solve_cg(G12, B, X12, dims, kappa, tol=1e-10,
                                                maxiter=20000, flags=f, work=wk, stream=s),
                             torch)
            assert st12["status"] == 0 and st12["true_res"] <= 1e-10, st12
            link12_solves[name] = {"seconds": dt, "iterations": st12["iterations"],
                                   "true_res": st12["true_res"],
                                   "speedup_vs_18_real": ref / dt if ref else None}
            del wk
        del G12, X12

    # the twisted-mass operator of the paper's action, mu = 0.01, with the
    # step's solver (mixed-precision eo-CG); the twist bounds sigma_min(M)
    # from below by 2 kappa mu, so it converges in fewer iterations
    tm_solve = None
    if not args.no_fp64_compare:
        mu = 0.01
        wk = torch.empty(w.workspace_bytes(dims, flags), dtype=torch.uint8, device="cuda")
        Xt = w.empty_spinor(dims)
        w.solve_cg_tm(G64, B, Xt, dims, kappa, mu, tol=1e-10, maxiter=20000, flags=flags,
                      work=wk, stream=s)
        stt, dt = timed(lambda: w.solve_cg_tm(G64, B, Xt, dims, kappa, mu, tol=1e-10,
                                              maxiter=20000, flags=flags, work=wk, stream=s),
                        torch)
        assert stt["status"] == 0 and stt["true_res"] <= 1e-10, stt
        tm_solve = {"mu": mu, "seconds": dt, "iterations": stt["iterations"],
                    "true_res": stt["true_res"], "algorithmic_GBs": stt["bytes"] / dt / 1e9}
        del wk, Xt

    # Dslash variants, each timed over a run of launches (HIP events)
    variants = {}
    n = args.kernel_launches
    for prec, pname in ((w.F64, "f64"), (w.F32, "f32"), (w.F16S, "f16s")):
        for lk, lname in ((w.LINK18, "18"), (w.LINK12, "12")):
            G = w.pack_gauge(U, dims, prec | lk)
            P = w.pack_spinor(b, dims, prec)
            O = w.empty_spinor(dims, prec)
            Oh = w.empty_spinor(dims, prec, 1)
            sb = SPINOR_BYTES[prec]
            lb = COMPLEX_BYTES[prec] * (6 if lk else 9)
            f = prec | lk
            tm = time_kernel(lambda: w.wilson_dslash(G, P, O, dims, kappa, flags=f, stream=s),
                             n, torch)
            # beside the algorithmic rate, the paper's no-reuse convention: 8
            # neighbour spinors and 8 links read and one spinor written per
            # output site (2880 B for FP64-18), to compare with its 105 GB/s
            noreuse = 9 * sb + 8 * lb
            variants["M_%s_%s" % (pname, lname)] = {
                "us": tm * 1e6, "GBs": V * (2 * sb + 4 * lb) / tm / 1e9,
                "no_reuse_GBs": V * noreuse / tm / 1e9,
                "GFLOPs": 1368 * V / tm / 1e9}
            te = time_kernel(lambda: w.wilson_dslash_eo(
                G, w.parity_block(P, dims, prec, 0), Oh, dims, kappa, 1, flags=f | w.HOP,
                stream=s), n, torch)
            variants["Deo_%s_%s" % (pname, lname)] = {
                "us": te * 1e6, "GBs": Vh * (2 * sb + 8 * lb) / te / 1e9,
                "no_reuse_GBs": Vh * noreuse / te / 1e9,
                "GFLOPs": 1320 * Vh / te / 1e9}
            del G, P, O, Oh
    torch.cuda.empty_cache()

    # achievable bandwidth of a plain device copy of known size (also the
    # reference the profiler's byte counters are scaled by)
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    tc = time_kernel(lambda: dst.copy_(src), 20, torch)
    ts = time_kernel(lambda: w.stream_copy(src, dst, nbytes, stream=s), 20, torch)
    copy = {"bytes_moved": 2 * nbytes, "us": tc * 1e6, "GBs": 2 * nbytes / tc / 1e9,
            "stream_copy_us": ts * 1e6, "stream_copy_GBs": 2 * nbytes / ts / 1e9}
    best_copy = max(copy["GBs"], copy["stream_copy_GBs"])
    del src, dst

    # roofline of the dominant kernel of the step: the FP32 even-odd hop
    dom = "Deo_f32_%s" % ("12" if args.link12 else "18")
    lb = 8 * (6 if args.link12 else 9)
    per_launch = Vh * (2 * 96 + 8 * lb)
    ach = variants[dom]["GBs"]
    traffic = profiled_traffic(args.link12) if args.workload == "32^3x64" else None
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "wl::hop_kernel<float, %d, false, false, 0, 1, true> (even-odd hop, FP32)"
                          % (6 if args.link12 else 9),
                "bytes_per_launch": per_launch, "avg_us": variants[dom]["us"],
                "frac_of_copy": ach / best_copy}

    # the paper's measured kernel (Sec. 3, Fig. 5): the FP64 even-odd hop
    dom64 = "Deo_f64_%s" % ("12" if args.link12 else "18")
    lb64 = 16 * (6 if args.link12 else 9)
    per64 = Vh * (2 * 192 + 8 * lb64)
    roofline64 = {"bound": "hbm", "achieved": variants[dom64]["GBs"], "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": variants[dom64]["GBs"] / HBM_PEAK_GBS,
                  "traffic": (profiled_traffic(args.link12, fp64=True)
                              if args.workload == "32^3x64" else None),
                  "kernel": "wl::hop_kernel<double, %d, false, false, 0, 1, true> "
                            "(even-odd hop, FP64)" % (6 if args.link12 else 9),
                  "bytes_per_launch": per64, "avg_us": variants[dom64]["us"],
                  "gflops": variants[dom64]["GFLOPs"],
                  "no_reuse_GBs": variants[dom64]["no_reuse_GBs"]}

    small = None if args.no_small else small_configs(w, torch, synth, args.kernel_launches)

    gauge = None if args.no_small else pure_gauge(w, torch, synth, np, U, dims,
                                                   args.kernel_launches)

    batch = uneven = None
    if not args.no_batch:
        del G64, B, X, work
        torch.cuda.empty_cache()
        t = time.time()
        batch = batch12(w, torch, synth, args.kernel_launches)
        uneven = uneven64(w, torch, synth, np)
        log("batch measurements in %.1f s" % (time.time() - t))

    serve = None
    if not args.no_serving:
        torch.cuda.empty_cache()
        t = time.time()
        serve = serving(w, torch, synth, np, args.serving_requests, args.serving_budget_gb,
                        args.serving_slots, args.serving_merge)
        log("serving measurements in %.1f s" % (time.time() - t))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ncores = len(os.sched_getaffinity(0))
        oracle.set_threads(ncores)
        nrep = 2
        oracle.mop(U, b, dims, kappa)        # warm-up
        t = time.perf_counter()
        for _ in range(nrep):
            oracle.mop(U, b, dims, kappa)
        dt = (time.perf_counter() - t) / nrep
        # the step's own method on the host: a bounded number of the oracle's
        # FP64 even-odd CGNR iterations on the same system (the tolerance is
        # out of reach, so exactly `its` iterations run), counted with the
        # library's byte model of an FP64 eo-CG iteration (2 Schur applies of
        # 2 half hops, 1536 B per output site each, plus the xpay read, and 9
        # vector passes): Vh * (2 * (2 * 1536 + 192) + 9 * 192) bytes
        its = 30
        t = time.perf_counter()
        _, ost = oracle.cgnr_eo(U, b, dims, kappa, tol=1e-30, maxiter=its)
        dt_cg = time.perf_counter() - t
        iter_bytes = Vh * (2 * (2 * 1536 + 192) + 9 * 192)
        cpu = {"value": iter_bytes * ost["iterations"] / dt_cg / 1e9, "unit": "GB/s",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": "%d iterations of the oracle's FP64 even-odd CGNR on the %s "
                         "lattice (%.1f s; %.0f MB per iteration in the GPU solver's byte "
                         "model); the oracle's M apply on the same field: %.2f s, %.2f "
                         "GFLOP/s at 1368 flop/site" % (ost["iterations"], args.workload, dt_cg,
                                                         iter_bytes / 1e6, dt,
                                                         1368.0 * V / dt / 1e9),
               "seconds_per_iteration": dt_cg / max(ost["iterations"], 1),
               "seconds_per_apply": dt}
        # one host thread on the same apply; the M apply of the 4^4 and
        # 16^3 x 32 configurations (median of 10 / 3) and their CGNR solves to
        # 1e-10 (about 10 s of host time at 16^3 x 32), all threads
        oracle.set_threads(1)
        t = time.perf_counter()
        oracle.mop(U, b, dims, kappa)
        cpu["seconds_per_apply_1_core"] = time.perf_counter() - t
        oracle.set_threads(ncores)
        small_cpu = {}
        for name, d, kap, field, reps, solve in (
                ("4^4", (4, 4, 4, 4), 0.12, synth.gauge_haar((4, 4, 4, 4), 0), 10, True),
                ("16^3x32", (16, 16, 16, 32), 0.15, synth.gauge_smooth((16, 16, 16, 32), 0.30, 0),
                 3, True)):
            src = synth.gaussian_spinor(d, 1)
            ts = []
            for _ in range(reps):
                t = time.perf_counter()
                oracle.mop(field, src, d, kap)
                ts.append(time.perf_counter() - t)
            small_cpu[name] = {"M_apply_us": 1e6 * float(np.median(ts))}
            if solve:
                t = time.perf_counter()
                _, ost = oracle.cgnr(field, src, d, kap, tol=1e-10)
                small_cpu[name].update({"cgnr_seconds": time.perf_counter() - t,
                                        "cgnr_iterations": ost["iterations"],
                                        "cgnr_true_res": ost["true_res"]})
        cpu["small_configs"] = small_cpu

    detail = {
        "fp64_solve": fp64,
        "mixed_f16_solve": f16,
        "link12_solves": link12_solves,
        "twisted_mass_solve": tm_solve,
        "pure_gauge": gauge,
        "dslash_variants": variants,
        "device_copy": copy,
        "roofline": roofline,
        "roofline_fp64_eo": roofline64,
        "cpu_baseline": cpu,
        "small_configs": small,
        "batch12_point_sources": batch,
        "uneven64_lattices": uneven,
        "serving": serve,
    }
    # the details go to stderr and to a file; stdout ends with one compact line
    log("detail: " + json.dumps(detail))
    detail_path = os.path.join(ROOT, args.detail)
    os.makedirs(os.path.dirname(detail_path) or ROOT, exist_ok=True)
    with open(detail_path, "w") as f:
        json.dump(detail, f, indent=1)

    def pick(d, *keys):
        return None if d is None else {k: d[k] for k in keys if k in d}

    serve_sum = None
    if serve:
        serve_sum = {
            "mixed_saturation": serve["saturation_solves_per_s"],
            "fp64_saturation": serve["fp64_saturation_solves_per_s"]}
        for key, name in (("open_loop_0.5S", "mixed_0.5S"), ("open_loop_0.8S", "mixed_0.8S"),
                          ("open_loop_0.5S_edf", "mixed_0.5S_edf"),
                          ("open_loop_0.8S_edf", "mixed_0.8S_edf"),
                          ("mixed_at_0.5S64", "mixed_at_0.5S64"),
                          ("fp64_open_loop_0.5S64", "fp64_0.5S64"),
                          ("fp64_open_loop_0.8S64", "fp64_0.8S64")):
            r = serve[key]
            serve_sum[name] = [round(r["offered_rate"], 1), round(r["solves_per_s"], 1),
                               round(r["p50_ms"], 1), round(r["p99_ms"], 1)]
        serve_sum["fields"] = "offered req/s, solves/s, p50 ms, p99 ms"
    out = {
        "metric": "Dslash GB/s (% HBM peak) & GFLOP/s; solves/s + p99 latency, mixed vs FP64",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "wilson eo-CG mixed-precision solve %s" % args.workload,
                   "lattice": list(dims), "kappa": kappa, "links": "exp(i*%.2f*H), seed 0" % eps,
                   "link_storage": "12-real" if args.link12 else "18-real",
                   "tol": 1e-10, "parallelism": "single GPU"},
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "gflops": round(step_flops / (ms / 1e3) / 1e9, 1),
        "solves_per_s": round(1e3 / ms, 3),
        "iterations": int(np.mean([st["iterations"] for st in stats])),
        "true_res": max(st["true_res"] for st in stats),
        "fp64_solve_s": None if fp64 is None else round(fp64["seconds"], 4),
        "mixed_vs_fp64": None if fp64 is None else round(fp64["mixed_speedup"], 3),
        "f16_inner_solve_s": None if f16 is None else round(f16["seconds"], 4),
        "roofline": pick(roofline, "bound", "achieved", "peak", "unit", "frac", "traffic",
                         "kernel", "bytes_per_launch", "avg_us"),
        "roofline_fp64_eo": pick(roofline64, "bound", "achieved", "peak", "unit", "frac",
                                 "traffic", "kernel", "bytes_per_launch", "avg_us", "gflops",
                                 "no_reuse_GBs"),
        "cpu_baseline": pick(cpu, "value", "unit", "cores", "kind", "sample",
                             "seconds_per_iteration", "seconds_per_apply",
                             "seconds_per_apply_1_core"),
        "serving": serve_sum,
        "detail_file": args.detail,
    }
    for k in ("roofline", "roofline_fp64_eo"):
        if out[k]:
            for f in ("achieved", "frac", "avg_us", "gflops", "no_reuse_GBs"):
                if f in out[k]:
                    out[k][f] = round(out[k][f], 4)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
