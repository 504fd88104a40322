"""Serving loop for wave simulations on one GPU: continuous batching by quanta.

Requests (immersed-void problems of different geometries, sizes, degrees and step
counts) arrive over time.  The loop

* admits a waiting request when a slot is free and its device footprint fits the
  memory budget; admission runs the FP64 setup of the problem (classification, space
  tree quadrature, eigenvalue stabilisation, lumping, Lanczos critical step) on a
  set-up stream from a background thread (``setup_workers`` of them, each with its own
  stream), so set-ups overlap each other and the stepping of the problems already
  resident;
* keeps every admitted problem's fields resident on the device and advances all of
  them by one quantum of steps per round: problems of one kind (dimension, components,
  p; one precision) share one fused launch per step through fcw_run, the kinds follow
  one another on the same stream;
* retires a problem when its steps are done (its latency is completion - arrival) and
  frees its memory, so waiting requests can join at the next quantum boundary.

Every compute step runs in libfcw.so; this module only schedules calls.
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import threading
import time
from dataclasses import dataclass

import numpy as np

from . import fcw


@dataclass
class Request:
    rid: int
    cfg: dict                 # problem description (keys as in workloads.config)
    nsteps: int
    arrival: float = 0.0      # seconds after the start of the run
    sources: list = None      # one point source per right-hand side
    # filled by the server
    admitted: float = None
    dt: float = None
    setup_s: float = None     # wall time of its set-up (classification .. critical step)
    done: float = None
    dofs: int = 0
    state: object = None      # final u (host copy) when keep_results


@dataclass
class _Resident:
    req: Request
    ctx: object
    u: object
    d: object
    dt: float
    steps_done: int = 0
    footprint: int = 0


def estimate_footprint(cfg, nrhs=1, precision="fp32"):
    """Device bytes a problem needs before setup (upper estimate used for admission)."""
    dim, p = cfg["dim"], cfg["p"]
    ncomp = cfg.get("ncomp", 1)
    nc = int(np.prod(cfg["ncells"]))
    nn = int(np.prod([n * p + 1 for n in cfg["ncells"]]))
    s = 8 if precision == "fp64" else 4
    ns = (p + 1) ** dim
    nl = ncomp * ns
    ncut = nc  # worst case: every cell cut
    # state u, d, scratch; masses; per-cut-cell FP64 matrices and the packed copy
    b = 3 * nrhs * ncomp * nn * s + nn * (16 + s) + nc * 9
    b += min(ncut, max(1, nc // 4)) * (nl * nl * 8 + ns * ns * 8 + nl * (nl + 1) // 2 * s)
    return int(b)


class Server:
    def __init__(self, precision="fp32", device="cuda:0", memory_budget=None, max_slots=64,
                 quantum=100, keep_results=False, graph=True, setup_workers=2):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        self.stream = torch.cuda.Stream(self.device)
        # one set-up stream per worker thread, handed out from a free list
        self._setup_streams = [torch.cuda.Stream(self.device) for _ in range(setup_workers)]
        self._free_streams = list(self._setup_streams)
        self._streams_lock = threading.Lock()
        free, total = torch.cuda.mem_get_info(self.device)
        self.budget = int(memory_budget if memory_budget is not None else 0.8 * free)
        self.max_slots = max_slots
        self.quantum = quantum
        self.keep_results = keep_results
        self.graph = graph
        self._pool = cf.ThreadPoolExecutor(max_workers=setup_workers)

    # -- setup on the side stream (background thread) --
    def _setup(self, req):
        with self._streams_lock:
            stream = self._free_streams.pop()
        try:
            return self._setup_on(req, stream)
        finally:
            with self._streams_lock:
                self._free_streams.append(stream)

    def _setup_on(self, req, setup_stream):
        torch = self.torch
        t_setup = time.perf_counter()
        with torch.cuda.device(self.device):
            ctx = fcw.assemble_cells(req.cfg, self.precision,
                                     stream=setup_stream.cuda_stream)
            try:
                fcw.stabilize_cut_cells(ctx, req.cfg.get("eps", 1e-4),
                                        req.cfg.get("f_lambda", 1e-4))
                dtc = fcw.critical_dt(ctx, 4000, 1e-7)
                info = fcw.query(ctx)
                nrhs = len(req.sources)
                dtype = torch.float64 if self.precision == "fp64" else torch.float32
                with torch.cuda.stream(setup_stream):
                    u = torch.zeros(nrhs, info["ndof"], dtype=dtype, device=self.device)
                    d = torch.zeros_like(u)
                setup_stream.synchronize()
                u.record_stream(self.stream)
                d.record_stream(self.stream)
                # stepping goes on the serving stream; set-up of later requests keeps the
                # side stream
                fcw.set_stream(ctx, self.stream.cuda_stream)
            except Exception:
                fcw.destroy(ctx)
                raise
        fp = info["footprint_bytes"] + 3 * u.numel() * u.element_size()
        req.dofs = int(info["ndof"]) * nrhs
        req.setup_s = time.perf_counter() - t_setup
        # the step size comes from the library's rule (dt <= 0 in fcw_run) on the first
        # quantum and is kept for the later ones
        return _Resident(req=req, ctx=ctx, u=u, d=d, dt=None, footprint=fp)

    def run(self, requests, time_scale=1.0, log=None, log_every=20.0):
        """Serve ``requests`` (arrival times in seconds); returns a metrics dict.  ``log``, if
        given, is called with a one-line status about every ``log_every`` seconds."""
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting, resident, finished = [], [], []
        setting_up = {}        # future -> (request, reserved bytes)
        reserved = 0
        t_start = time.perf_counter()
        now = lambda: (time.perf_counter() - t_start) / time_scale
        total_updates = 0
        max_resident = peak_reserved = quanta = 0
        step_s = 0.0
        pi = 0
        next_log = log_every
        while pi < len(pending) or waiting or resident or setting_up:
            t = now()
            if log is not None and t >= next_log:
                log(f"t={t:.0f} s: {len(finished)}/{len(pending)} finished, {len(resident)} "
                    f"resident, {len(setting_up)} in set-up, {len(waiting)} waiting")
                next_log = t + log_every
            while pi < len(pending) and pending[pi].arrival <= t:
                waiting.append(pending[pi])
                pi += 1
            # admission: slot and memory permitting, in arrival order
            while waiting and len(resident) + len(setting_up) < self.max_slots:
                req = waiting[0]
                need = estimate_footprint(req.cfg, len(req.sources), self.precision)
                if reserved + need > self.budget and (resident or setting_up):
                    break
                waiting.pop(0)
                reserved += need
                req.admitted = t
                setting_up[self._pool.submit(self._setup, req)] = (req, need)
                peak_reserved = max(peak_reserved, reserved)
            # problems whose setup finished join at this quantum boundary
            for fut in [f for f in setting_up if f.done()]:
                req, need = setting_up.pop(fut)
                res = fut.result()
                reserved += res.footprint - need
                resident.append(res)
            if not resident:
                if setting_up:
                    cf.wait(list(setting_up), timeout=0.05, return_when=cf.FIRST_COMPLETED)
                elif pi < len(pending):
                    time.sleep(max(0.0, min(0.05, (pending[pi].arrival - now()) * time_scale)))
                continue
            # one quantum for every resident problem, fused by kind
            max_resident = max(max_resident, len(resident))
            quanta += 1
            t_q = time.perf_counter()
            groups = {}
            for r in resident:
                c = r.req.cfg
                key = (c["dim"], c.get("ncomp", 1), c["p"])
                groups.setdefault(key, []).append(r)
            with torch.cuda.stream(self.stream):
                for key, members in groups.items():
                    entries = []
                    for r in members:
                        n = min(self.quantum, r.req.nsteps - r.steps_done)
                        dt_max = r.req.cfg.get("dt_max", math.inf)
                        entries.append(dict(ctx=r.ctx, nrhs=len(r.req.sources), u=r.u, d=r.d,
                                            sources=r.req.sources,
                                            t0=r.steps_done * r.dt if r.dt else 0.0,
                                            dt=r.dt or 0.0,
                                            dt_max=dt_max if math.isfinite(dt_max) else 0.0,
                                            nsteps=n, start=int(r.steps_done == 0)))
                    # one kind per call: the library advances the members together
                    outs = fcw.run(entries, graph=self.graph)
                    for r, o in zip(members, outs):
                        r.dt = r.req.dt = o["dt_used"]
            self.stream.synchronize()
            step_s += time.perf_counter() - t_q
            t = now()
            still = []
            for r in resident:
                n = min(self.quantum, r.req.nsteps - r.steps_done)
                r.steps_done += n
                total_updates += r.req.dofs * n
                if r.steps_done >= r.req.nsteps:
                    r.req.done = t
                    if self.keep_results:
                        r.req.state = r.u.cpu().numpy().copy()
                    fcw.destroy(r.ctx)
                    reserved -= r.footprint
                    finished.append(r.req)
                else:
                    still.append(r)
            resident = still
        makespan = now()
        lat = np.array([r.done - r.arrival for r in finished])
        setup = np.array([r.setup_s for r in finished])
        return dict(n=len(finished), makespan_s=makespan, quanta=quanta,
                    setup_s_total=float(setup.sum()) if len(setup) else 0.0,
                    setup_s_max=float(setup.max()) if len(setup) else 0.0,
                    stepping_s=step_s,
                    max_resident=max_resident, peak_reserved_bytes=peak_reserved,
                    dof_updates_per_s=total_updates / max(makespan, 1e-12),
                    p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else None,
                    p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else None,
                    mean_latency_s=float(lat.mean()) if len(lat) else None)

    def close(self):
        self._pool.shutdown(wait=True)


def requests_from_stream(stream, scale=1.0, precision_eps=1e-4):
    """Turn workloads.request_stream records into Requests (sizes scaled by ``scale``)."""
    import workloads
    out = []
    for r in stream:
        dim = r["dim"]
        n = max(4, int(round(r["n"] * scale)))
        if dim == 2:
            cc, rr = workloads.random_circles(seed=r["void_seed"], count=40)
        else:
            cc, rr = workloads.random_spheres(seed=r["void_seed"], n_probe=20000)
        cfg = workloads._base(dim, (n,) * dim, r["p"], cc, rr, nsteps=r["nsteps"],
                              eps=precision_eps)
        src = [dict(x=(0.1,) * dim, dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)]
        out.append(Request(rid=r["id"], cfg=cfg, nsteps=r["nsteps"], arrival=r["arrival"],
                           sources=src))
    return out
