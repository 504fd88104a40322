"""Convenience wrapper of the fcw C ABI with torch device memory and streams.

Marshalling only: the context, the stiffness products and the updates all live in
libfcw.so.  torch provides the device buffers (state vectors) and the stream.
"""
from __future__ import annotations

from . import fcw


class Solver:
    """One immersed problem on one GPU: assemble, stabilise, dt, step."""

    def __init__(self, cfg, precision="fp32", device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cfg = cfg
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        with torch.cuda.device(self.device):
            self.ctx = fcw.assemble_cells(cfg, precision, stream=self.stream.cuda_stream)
            fcw.stabilize_cut_cells(self.ctx, cfg.get("eps", 1e-4), cfg.get("f_lambda", 1e-4))
        self.info = fcw.query(self.ctx)

    @property
    def ndof(self):
        return self.info["ndof"]

    def critical_dt(self, max_iter=4000, rtol=1e-9):
        dtc = fcw.critical_dt(self.ctx, max_iter, rtol)
        self.info = fcw.query(self.ctx)
        return dtc

    def autotune(self, nrhs=1, nsteps=20):
        """Pick the fastest compiled tile configuration of the step for this problem."""
        chosen, table = fcw.autotune(self.ctx, nrhs, nsteps)
        return chosen, table

    def select_tile(self, i):
        fcw.select_tile(self.ctx, i)

    def tile_configs(self):
        return fcw.tile_configs(self.ctx)

    def zeros(self, nrhs=1):
        return self.torch.zeros(nrhs, self.ndof, dtype=self.dtype, device=self.device)

    def step(self, u, d, sources, dt, nsteps, t0=0.0, start=False):
        """Advance (u, d) in place; ``sources``: list of dicts, one per right-hand side."""
        nrhs = u.shape[0] if u.dim() == 2 else 1
        fcw.step_explicit(self.ctx, nrhs, u, d, sources, t0, dt, nsteps, 1 if start else 0)

    def run(self, sources, dt, nsteps, nrhs=None, u=None, d=None):
        """Zero initial state, ``nsteps`` steps from t = 0 with the Newmark start-up."""
        nrhs = nrhs or (len(sources) if sources else 1)
        u = self.zeros(nrhs) if u is None else u
        d = self.zeros(nrhs) if d is None else d
        self.step(u, d, sources, dt, nsteps, 0.0, True)
        return u, d

    def apply_stiffness(self, u):
        r = self.torch.empty_like(u)
        nrhs = u.shape[0] if u.dim() == 2 else 1
        fcw.apply_stiffness(self.ctx, nrhs, u, r)
        return r

    def export(self, which):
        return fcw.export(self.ctx, which)

    def close(self):
        if self.ctx:
            fcw.destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

