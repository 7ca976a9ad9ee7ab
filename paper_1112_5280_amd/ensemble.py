"""A Markov chain of gauge configurations with a measurement on each: the
hybrid task split of paper Sec. 4 (Fig. 6/7), where one device generates the
next configuration while another measures the current one.

On one MI355X the two tasks are two HIP streams: the heat-bath sweeps that
turn configuration k into k+1 are enqueued on the generation stream, and the
measurement of configuration k (the 12 point-source solves of one
propagator, the meson correlators of Eq. 1) runs meanwhile on the measurement
stream. Configurations stay in the packed FP64 layout the solvers read (the
heat bath on that layout is bitwise the one on the canonical field), so
nothing is packed between the update and the measurement. Every step is a library call; this module only orders them (events
between the streams) and holds the buffers. The chain and the measurements do
not depend on the overlap: the kernels are deterministic and each link's
random numbers are fixed by (seed, sweep, site, direction)."""
from __future__ import annotations

import time

import numpy as np
import torch

from . import wilson as w


class Ensemble:
    """Configurations U_0 (given) -> U_1 -> ... by `sweeps` heat-bath sweeps at
    coupling beta each; on every configuration the propagator of the 12 point
    sources at `site` is solved (batched even-odd CG, `flags`) and its 16 meson
    correlators are formed. `run(n)` returns the correlators [n, 16, Lt]."""

    def __init__(self, U0, dims, beta, sweeps, kappa, site, seed=0, flags=w.EO, tol=1e-10,
                 maxiter=20000, overlap=True):
        self.dims = tuple(dims)
        self.beta, self.sweeps, self.kappa, self.seed = beta, sweeps, kappa, seed
        self.flags, self.tol, self.maxiter, self.overlap = flags, tol, maxiter, overlap
        self.site = int(site)
        V = int(np.prod(dims))
        self.t0 = self.site // (dims[0] * dims[1] * dims[2])
        dev = "cuda"
        G0 = w.pack_gauge(U0, dims)                  # packed FP64 18-real
        self.G = [G0, torch.empty_like(G0)]
        self.B = w.empty_batch(dims, 12)
        src = torch.zeros((V, 4, 3), dtype=torch.complex128, device=dev)
        for r in range(12):
            src.zero_()
            src[self.site, r // 3, r % 3] = 1.0
            w.pack_spinor(src, dims, out=w.batch_field(self.B, dims, 0, r))
        self.X = w.empty_batch(dims, 12)
        self.work = torch.empty(w.workspace_bytes(dims, flags, 12), dtype=torch.uint8,
                                device=dev)
        self.mwork = torch.empty(w.lib.wl_meson_workspace_bytes(w._dims(dims)),
                                 dtype=torch.uint8, device=dev)
        self.gen = torch.cuda.Stream()
        self.meas = torch.cuda.Stream() if overlap else self.gen
        # the buffers above were filled on the current stream
        self.gen.wait_stream(torch.cuda.current_stream())
        self.meas.wait_stream(torch.cuda.current_stream())
        self.sweep = 0
        self.stats = []

    @property
    def U(self):
        """The two configurations held (k % 2 holds configuration k), as
        canonical complex128 fields [V, 4, 3, 3] (exact copies)."""
        return [w.unpack_gauge(g, self.dims) for g in self.G]

    def _generate(self, k):
        """G[(k+1)%2] = heat bath of G[k%2], enqueued on the generation stream."""
        src, dst = self.G[k % 2], self.G[(k + 1) % 2]
        with torch.cuda.stream(self.gen):
            dst.copy_(src)
            w.heatbath_packed(dst, self.dims, self.beta, self.sweeps, self.sweep, self.seed,
                              stream=self.gen)
        self.sweep += self.sweeps

    def _measure(self, k):
        """Correlators of configuration k on the measurement stream."""
        s = self.meas
        code, st = w.solve_cg_batch(self.G[k % 2], self.B, self.X, 12, self.dims, self.kappa,
                                    tol=self.tol, maxiter=self.maxiter, flags=self.flags,
                                    work=self.work, stream=s)
        if code != w.OK:
            raise w.WilsonError(code, "propagator solve of configuration %d" % k)
        self.stats.append(st)
        return w.meson_correlators(self.X, self.dims, self.t0, work=self.mwork, stream=s)

    def run(self, n):
        out = []
        ready = torch.cuda.Event()
        for k in range(n):
            self.meas.wait_stream(self.gen)      # configuration k is complete
            if self.overlap:
                # configuration k+1 needs k intact until it has copied it; the
                # measurement only reads G[k % 2], the sweeps write G[(k+1) % 2]
                self._generate(k)
                corr = self._measure(k)
            else:
                corr = self._measure(k)
                self._generate(k)
            ready.record(self.meas)
            ready.synchronize()
            out.append(corr.cpu())
            # the next generation overwrites G[k % 2]: wait for this measurement
            self.gen.wait_stream(self.meas)
        self.gen.synchronize()
        return torch.stack(out)
