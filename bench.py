#!/usr/bin/env python3
"""Benchmark of the explicit spectral-cell wave step on one MI355X.

Workload: 2-D scalar wave on [0,1]^2 with 40 random circular voids (radii 0.01-0.05,
seed 2), 512 x 512 cells, p = 4 GLL (about 4.2 M DOF), Ricker point source f0 = 10 at
(0.1, 0.1), dt = 0.9 dt_crit, eps = 1e-4 eigenvalue stabilisation, FP64 setup; the
stiffness product and the state run in FP32 (matrix cores) and, for reference, in FP64.

A step is one central-difference step of the whole hot path (uncut MFMA contraction,
cut-cell stream, gather, lumped-mass update) over one right-hand side.  `value` is
DOF-updates/s of the FP32 path: active DOFs x steps / stepping time, measured with HIP
events on the solver's stream around exactly --steps steps (inputs resident in HBM).
The FP32 result is compared with the FP64 GPU path after the same steps (relative L2
over all DOFs, `rel_l2_vs_fp64`) and, from the cpu_baseline leg, both forms with the
oracle (`rel_l2_vs_oracle`).

Roofline: a step is two kernels, the cut-cell product kernel (it streams the packed
cut-cell matrices, N_cut (n_loc(n_loc+1)/2 s + 4) bytes) and the main step kernel (the
state: 3 s N_dof + s N_cutadj + N_cells / 8 bytes -- read u_k and u_{k-1}, write u_{k+1};
the non-analytic inverse masses next to cut cells; one class bit per cell).  Each
kernel's algorithmic bytes are divided by its own average launch duration, measured with
HIP events around one replay of a captured graph of --steps launches of that kernel back
to back (fcw_kernel_times), against 8 TB/s of HBM3E; `roofline` reports the main kernel, which
dominates the step time.  The main kernel is also priced against the matrix cores (the
uncut contraction, 2 n_loc^2 flops per uncut cell, at the dense peak of its operand
type); `bound` names the roofline whose time at peak is longer (HBM for the 2-D workload;
the matrix cores for the FP32 3-D elastic one), the other sits under `other`.

cpu_baseline: the FP64 oracle stepping the same full-size problem for a bounded number of
steps on the host, on every thread torch uses and on one thread, at its own dt = 0.9 dt_crit;
the FP32 and FP64 device states after the same steps from rest at that dt are compared with
the oracle's (`rel_l2_vs_oracle`).

Further legs in the same JSON line: `c3` (3-D elastic 96^3 p=2: FP32, split BF16, FP64),
`imex` (the semi-explicit scheme of Alg. imex, FP64, on the same void field at 64^2 p=3
and at its full size),
`iga` (IGA-FCM with B-splines and row-sum lumping on the 512^2 void field, p=4, FP32) and
`serving` (p50/p99 latency of a seeded request stream).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of MI355X by operand type (TFLOP/s)
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6}


def algorithmic_bytes(cfg, info, cls, s_state, part="step"):
    """Per-step algorithmic bytes (see module docstring).  part="main": the state terms
    moved by the main step kernel; part="cut": the packed cut-cell matrices streamed by
    the cut-cell kernel; "step": both."""
    p, dim = cfg["p"], cfg["dim"]
    ncells = np.array(cfg["ncells"])
    nl = info["n_loc"]
    n_dof = info["ndof"]
    # nodes touched by at least one cut cell
    grid = cls.reshape(tuple(ncells[::-1]))
    cut = (grid == 2)
    npts = ncells * p + 1
    mark = np.zeros(tuple(npts[::-1]), dtype=bool)
    if dim == 2:
        cy, cx = np.nonzero(cut)
        for a in range(p + 1):
            for b in range(p + 1):
                mark[cy * p + a, cx * p + b] = True
    else:
        cz, cy, cx = np.nonzero(cut)
        for a in range(p + 1):
            for b in range(p + 1):
                for c in range(p + 1):
                    mark[cz * p + a, cy * p + b, cx * p + c] = True
    n_cutadj = int(mark.sum()) * cfg.get("ncomp", 1)
    n_cut = info["n_cut"]
    main = 3 * s_state * n_dof + s_state * n_cutadj + int(np.prod(ncells)) / 8.0
    cut = n_cut * (nl * (nl + 1) // 2 * s_state + 4)
    return {"main": main, "cut": cut, "step": main + cut}[part]


def run_gpu(cfg, precision, steps, warmup, dt=None):
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver

    s = Solver(cfg, precision=precision, device="cuda:0")
    if dt is None:
        dt = 0.9 * s.critical_dt(max_iter=4000, rtol=1e-7)
    src = cfg["sources"]
    chosen, table = s.autotune(nrhs=1, nsteps=30)
    print(f"[bench] {precision} autotune: " + ", ".join(
        f"{t['tile']}:{t['us_per_step']:.1f}us" for t in table) + f" -> {table[chosen]['tile']}",
        file=sys.stderr, flush=True)
    u, d = s.zeros(1), s.zeros(1)
    if warmup:
        s.step(u, d, src, dt, warmup, t0=0.0, start=True)
    stream = s.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(u, d, src, dt, steps, t0=warmup * dt, start=(warmup == 0))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # per-kernel launch durations: each kernel timed over `steps` launches back to back
    # with HIP events on the solver's stream, on the library's scratch state
    main_us, cut_us = fcw.kernel_times(s.ctx, 1, steps)
    cls = s.export(fcw.ARR_CELL_CLASS)
    mass = s.export(fcw.ARR_MASS)
    info = dict(s.info)
    out = u[0].double().cpu().numpy()
    s.close()
    return dict(ms=ms, steps=steps, dt=dt, info=info, cls=cls, active=int((mass > 0).sum()) * cfg.get("ncomp", 1),
                u=out, tile=table[chosen]["tile"], kernel=table[chosen]["kernel"],
                main_ms=main_us * 1e-3, main_launches=steps,
                cut_ms=cut_us * 1e-3, cut_launches=steps if cut_us > 0 else 0,
                cut_kernel="fcw::cut_apply_kernel<%s, %d, %d, %d, true>" % (
                    "double" if precision == "fp64" else "float", cfg["dim"], cfg["p"],
                    cfg.get("ncomp", 1)))


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed counter summaries under
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when none
    was taken or the kernel's sources have changed since (each summary names the files
    its sha1 covers)."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            lines = fh.read().splitlines()
        for i, line in enumerate(lines):
            if line.strip() != f"kernel: {kernel}":
                continue
            fields = {}
            for l2 in lines[i + 1:i + 4]:
                k, _, v = l2.partition(":")
                fields[k.strip()] = v.strip()
            if "traffic_bytes_per_launch" not in fields or "source_sha1" not in fields:
                continue
            sha, _, files = fields["source_sha1"].partition(" ")
            h = hashlib.sha1()
            names = files.strip("() ").replace("sha1 over ", "").split(", ")
            if not all(os.path.exists(os.path.join(ROOT, f)) for f in names):
                continue
            for f in names:
                with open(os.path.join(ROOT, f), "rb") as fh:
                    h.update(fh.read())
            if h.hexdigest() == sha:
                return float(fields["traffic_bytes_per_launch"])
    return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, nsteps_all, nsteps_one):
    """The FP64 oracle on the host: its own set-up and dt = 0.9 dt_crit (dt_crit from its
    eigen-solve), then ``nsteps_all`` steps timed on every host thread torch uses and
    ``nsteps_one`` steps on one thread.  Returns the baseline record, the oracle's dt and
    its state after ``nsteps_all`` steps (the parity reference of the bench line)."""
    import torch
    from threadpoolctl import threadpool_limits

    from oracle import problem, timestep
    t = time.perf_counter()
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = 0.9 * timestep.critical_dt(disc, tol=1e-10)
    t_setup = time.perf_counter() - t
    active = int((disc.mass > 0).sum()) * cfg.get("ncomp", 1)
    nthreads = torch.get_num_threads()
    t = time.perf_counter()
    ref = timestep.cdm(disc, dt, nsteps_all, sources=cfg["sources"])["u"]
    el_all = time.perf_counter() - t
    torch.set_num_threads(1)
    try:
        with threadpool_limits(limits=1):
            t = time.perf_counter()
            timestep.cdm(disc, dt, nsteps_one, sources=cfg["sources"])
            el_one = time.perf_counter() - t
    finally:
        torch.set_num_threads(nthreads)
    rec = dict(value=active * nsteps_all / el_all, unit="DOF-updates/s", cores=nthreads,
               kind="oracle",
               sample=f"{nsteps_all} steps of the full 512x512 p=4 problem from rest, FP64 "
                      f"numpy + torch CPU, {nthreads} threads, {el_all:.1f} s (set-up and the "
                      f"oracle's own dt_crit eigen-solve, {t_setup:.1f} s, excluded)",
               cpu=_cpu_model(),
               single_thread=dict(value=active * nsteps_one / el_one, cores=1,
                                  sample=f"{nsteps_one} steps, 1 thread, {el_one:.1f} s"))
    return rec, dt, ref


def gpu_state(cfg, precision, dt, nsteps):
    """The device state after ``nsteps`` steps from rest at step ``dt`` (autotuned kernel,
    as in the timed runs)."""
    import torch
    from paper_2501_19013_amd.solver import Solver
    s = Solver(cfg, precision=precision, device="cuda:0")
    s.autotune(nrhs=1, nsteps=30)
    u, d = s.zeros(1), s.zeros(1)
    s.step(u, d, cfg["sources"], dt, nsteps, t0=0.0, start=True)
    torch.cuda.synchronize()
    out = u[0].double().cpu().numpy()
    s.close()
    return out


def roofline(cfg, r, precision="fp32"):
    """Roofline of the dominant (main) step kernel from its own event-timed launches,
    plus the cut-cell kernel and the whole step.  The main kernel is priced against
    both HBM (its algorithmic bytes) and the matrix cores (the uncut contraction,
    2 n_loc^2 flops per uncut cell, at the dense peak of its operand type); `bound` is
    the one whose time at peak is longer, the other is reported under `other`."""
    Bm = algorithmic_bytes(cfg, r["info"], r["cls"], 4, "main")
    Bc = algorithmic_bytes(cfg, r["info"], r["cls"], 4, "cut")
    t = r["main_ms"] * 1e-3
    nl = r["info"]["n_loc"]
    F = 2.0 * nl * nl * int((np.asarray(r["cls"]) == 1).sum())
    pk = MFMA_PEAK_TFLOPS[precision]
    hbm = dict(bound="hbm", achieved=Bm / t / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
               frac=Bm / t / 1e9 / HBM_PEAK_GBS, algorithmic_bytes_per_launch=Bm)
    mfma = dict(bound="mfma", achieved=F / t / 1e12, peak=pk, unit="TFLOP/s",
                frac=F / t / 1e12 / pk, algorithmic_flops_per_launch=F)
    first, other = (mfma, hbm) if F / (pk * 1e12) > Bm / (HBM_PEAK_GBS * 1e9) else (hbm, mfma)
    out = dict(first, traffic=measured_traffic(r["kernel"]), kernel=r["kernel"],
               algorithmic_bytes_per_launch=Bm, avg_launch_ms=r["main_ms"],
               launches_timed=r["main_launches"], other=other)
    if r["cut_launches"]:
        ac = Bc / (r["cut_ms"] * 1e-3) / 1e9
        out["cut_kernel"] = dict(kernel=r["cut_kernel"], achieved=ac, frac=ac / HBM_PEAK_GBS,
                                 algorithmic_bytes_per_launch=Bc, avg_launch_ms=r["cut_ms"],
                                 launches_timed=r["cut_launches"])
    ms_step = r["ms"] / r["steps"]
    out["whole_step"] = dict(achieved=(Bm + Bc) / (ms_step * 1e-3) / 1e9,
                             frac=(Bm + Bc) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             algorithmic_bytes=Bm + Bc, ms=ms_step)
    return out


def bench_c3(steps, warmup, with_fp64):
    """3-D elastic workload: 96^3 cells, p=2, random spherical pores (porosity 0.2)."""
    import workloads
    cfg = workloads.config("c3")
    r32 = run_gpu(cfg, "fp32", steps, warmup)
    print(f"[bench] c3 fp32: {steps} steps in {r32['ms']:.2f} ms", file=sys.stderr, flush=True)
    ms_step = r32["ms"] / steps
    out = dict(workload="c3: 3-D elastic wave, unit cube, random spherical pores (porosity 0.2, "
                        "r 0.02-0.06, seed 3), 96^3 cells, p=2 GLL, 3 components, FP32 step, FP64 "
                        "setup, Ricker point force e_x at (0.1,0.1,0.1), dt=0.9 dt_crit",
               value=r32["active"] * steps / (r32["ms"] * 1e-3), unit="DOF-updates/s",
               ms_per_step=ms_step, steps=steps, warmup=warmup,
               ndof=r32["info"]["ndof"], active_dof=r32["active"], n_cut=r32["info"]["n_cut"],
               dt=r32["dt"], roofline=roofline(cfg, r32, "fp32"))
    rbf = run_gpu(cfg, "bf16", steps, warmup, dt=r32["dt"])
    print(f"[bench] c3 bf16: {steps} steps in {rbf['ms']:.2f} ms", file=sys.stderr, flush=True)
    out["bf16_split"] = dict(value=rbf["active"] * steps / (rbf["ms"] * 1e-3),
                             ms_per_step=rbf["ms"] / steps, roofline=roofline(cfg, rbf, "bf16"))
    if with_fp64:
        r64 = run_gpu(cfg, "fp64", steps, warmup, dt=r32["dt"])
        print(f"[bench] c3 fp64: {steps} steps in {r64['ms']:.2f} ms", file=sys.stderr, flush=True)
        out["fp64_gpu"] = dict(value=r64["active"] * steps / (r64["ms"] * 1e-3),
                               ms_per_step=r64["ms"] / steps)
        out["speedup_vs_fp64_gpu"] = out["value"] / out["fp64_gpu"]["value"]
        nrm = np.linalg.norm(r64["u"])
        out["rel_l2_vs_fp64"] = float(np.linalg.norm(r32["u"] - r64["u"]) / nrm)
        out["bf16_split"]["rel_l2_vs_fp64"] = float(np.linalg.norm(rbf["u"] - r64["u"]) / nrm)
        out["bf16_split"]["speedup_vs_fp64_gpu"] = out["bf16_split"]["value"] / out["fp64_gpu"]["value"]
    return out


def bench_c4(steps, warmup):
    """The 3-D elastic workload at 64^3 cells, p = 3 (n_loc = 192), with its 16 source
    positions as right-hand sides of one explicit FP32 run (the explicit part of the IMEX
    configuration; its implicit set is one block of millions of DOFs, beyond the dense
    block limit)."""
    import torch
    import workloads
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg = workloads.config("c4")
    # a source position inside a pore moves up in z until it is in the material
    cen = np.asarray(cfg["void_center"], dtype=float).reshape(-1, 3)
    rad = np.asarray(cfg["void_radius"], dtype=float)
    src = []
    for sd in cfg["sources"]:
        x = np.array(sd["x"], dtype=float)
        while np.any(np.linalg.norm(cen - x, axis=1) <= rad + 0.01):
            x[2] += 0.01
        src.append(dict(sd, x=tuple(float(v) for v in x)))
    t0 = time.perf_counter()
    s = Solver(cfg, precision="fp32", device="cuda:0")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = s.info
    print(f"[bench] c4 set-up {t_setup:.1f} s, {info['n_cut']} cut cells", file=sys.stderr,
          flush=True)
    s.autotune(nrhs=len(src), nsteps=3)
    dt = 0.9 * s.critical_dt(max_iter=4000, rtol=1e-7)
    u, d = s.zeros(len(src)), s.zeros(len(src))
    s.step(u, d, src, dt, warmup, t0=0.0, start=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(u, d, src, dt, steps, t0=warmup * dt, start=False)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    active = int((s.export(fcw.ARR_MASS) > 0).sum())
    ok = bool(torch.isfinite(u).all())
    s.close()
    return dict(workload="c4: 3-D elastic, the c3 pore field at 64^3 cells, p=3 GLL (192 DOFs "
                         "per cell), 16 source positions as right-hand sides, FP32 explicit "
                         "step, FP64 setup", value=len(src) * active * steps / (ms * 1e-3),
                unit="DOF-updates/s", ms_per_step=ms / steps, nrhs=len(src), steps=steps,
                ndof=info["ndof"], active_dof=active, n_cut=info["n_cut"], setup_s=t_setup,
                dt=dt, finite=ok)


def _imex_leg(cfg, steps, warmup, batch_rhs=0):
    """IMEX, explicit and consistent-mass steps of one FP64 problem, each timed over
    ``steps`` steps after ``warmup``; with ``batch_rhs`` also IMEX steps with that many
    right-hand sides."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    src = cfg["sources"][:1]
    s = Solver(cfg, precision="fp64", device="cuda:0")
    s.autotune(nrhs=1, nsteps=30)  # the explicit part's kernel, as for the explicit legs
    dt = 0.9 * s.critical_dt(max_iter=4000, rtol=1e-7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nc = fcw.imex_prepare(s.ctx, dt)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    lay = fcw.imex_layout(s.ctx)
    u, d = s.zeros(1), s.zeros(1)
    v = torch.zeros(1, max(nc, 1), dtype=torch.float64, device="cuda:0")
    a = torch.zeros_like(v)
    stream = s.stream
    fcw.step_imex(s.ctx, 1, u, d, v, a, src, 0.0, dt, warmup, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fcw.step_imex(s.ctx, 1, u, d, v, a, src, warmup * dt, dt, steps, 0)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    active = int((s.export(fcw.ARR_MASS) > 0).sum())
    # the explicit step alone on the same problem, for scale
    u2, d2 = s.zeros(1), s.zeros(1)
    s.step(u2, d2, src, dt, warmup, t0=0.0, start=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(u2, d2, src, dt, steps, t0=warmup * dt, start=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_exp = e0.elapsed_time(e1)
    # central differences with the consistent cut-DOF mass (its own, smaller stable step
    # is the caller's business; the cost per step does not depend on dt)
    u3, d3 = s.zeros(1), s.zeros(1)
    fcw.step_consistent(s.ctx, 1, u3, d3, src, 0.0, dt, warmup, 1)
    torch.cuda.synchronize()
    e0.record(stream)
    fcw.step_consistent(s.ctx, 1, u3, d3, src, warmup * dt, dt, steps, 0)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_con = e0.elapsed_time(e1)
    batch = {}
    if batch_rhs > 0:
        # batch_rhs source positions as right-hand sides of one run (the first points of a
        # 9 x 9 grid over the interior that lie in the material): each tile of S^-1 is read
        # once per step for all of them
        cen = np.asarray(cfg["void_center"], dtype=float).reshape(-1, 2)
        rad = np.asarray(cfg["void_radius"], dtype=float)
        srcs = []
        for iy in range(9):
            for ix in range(9):
                x = np.array([0.1 + 0.1 * ix, 0.1 + 0.1 * iy])
                if len(rad) == 0 or np.all(np.linalg.norm(cen - x, axis=1) > rad + 0.01):
                    srcs.append(dict(x=(float(x[0]), float(x[1])), f0=10.0, amp=1.0))
        srcs = srcs[:batch_rhs]
        batch_rhs = len(srcs)
        ub, db = s.zeros(batch_rhs), s.zeros(batch_rhs)
        vb = torch.zeros(batch_rhs, max(nc, 1), dtype=torch.float64, device="cuda:0")
        ab = torch.zeros_like(vb)
        fcw.step_imex(s.ctx, batch_rhs, ub, db, vb, ab, srcs, 0.0, dt, warmup, 1)
        torch.cuda.synchronize()
        e0.record(stream)
        fcw.step_imex(s.ctx, batch_rhs, ub, db, vb, ab, srcs, warmup * dt, dt, steps, 0)
        e1.record(stream)
        torch.cuda.synchronize()
        msb = e0.elapsed_time(e1)
        batch = dict(batch_rhs=batch_rhs, batch_ms_per_step=msb / steps,
                     batch_value=batch_rhs * active * steps / (msb * 1e-3))
    s.close()
    return dict(value=active * steps / (ms * 1e-3), unit="DOF-updates/s", ms_per_step=ms / steps,
                steps=steps, n_implicit=nc, n_blocks=lay["n_blocks"],
                largest_block=lay["largest"], active_dof=active, prepare_s=t_prep, dt=dt,
                explicit_ms_per_step=ms_exp / steps,
                consistent_mass_cdm_ms_per_step=ms_con / steps,
                # the packed upper tiles of the blocks of S^-1, read once per step
                solve_bytes_per_step=lay["solve_bytes"], **batch)


def bench_imex(steps, warmup, full_steps):
    """Semi-explicit (IMEX) scheme, FP64: the C2 void field at 64 x 64 cells, p = 3 (about
    5.7 k implicit DOFs), and at its full size, 512 x 512 cells, p = 4 (about 80 k implicit
    DOFs).  S and M^cc are block diagonal over the blocks of coupled implicit DOFs; each
    block is dense, factored and inverted once on the device."""
    import workloads
    cc, rr = workloads.random_circles(seed=2)
    cfg = workloads._base(2, (64, 64), 3, cc, rr, nsteps=steps)
    res = _imex_leg(cfg, steps, warmup)
    res["workload"] = ("2-D scalar, the c2 void field at 64x64 cells, p=3 GLL, FP64, IMEX "
                       "(Alg. imex, beta=1/4, gamma=1/2), S and M^cc block diagonal: dense "
                       "FP64 Cholesky per block, S^-1 as packed upper tiles")
    if full_steps > 0:
        full = _imex_leg(workloads.config("c2"), full_steps, warmup, batch_rhs=16)
        full["workload"] = "the same scheme on the c2 void field at full size, 512x512 cells, p=4"
        res["c2_full"] = full
    return res


def bench_iga(steps, warmup):
    """IGA-FCM (B-splines, row-sum lumped mass, central differences) on the c2 void field:
    512 x 512 cells, p = 4, 516^2 DOFs, FP32 steps with an FP64 run of the same steps for
    the relative L2 difference.  One launch per step (iga_step_kernel).  Algorithmic bytes
    per step: 5 s N_dof (read u_k, d_k, 1/m; write u_{k+1}, d_{k+1}) + N_cut n_s^2 s (the
    cut cells' matrices) + 4 N_cells (cell infos); flops: 2 n_s^2 per kept cell, on the
    FP32 vector units (157.3 TFLOP/s)."""
    import torch
    import workloads
    from paper_2501_19013_amd import fcw
    cfg = workloads.config("c2")
    src = cfg["sources"]
    out = dict(workload="c2 void field, IGA-FCM: maximum-continuity B-splines p=4 on 512x512 "
                        "cells (516^2 DOFs), row-sum lumped mass, alpha=1e-12, Ricker f0=10 at "
                        "(0.1,0.1), dt=0.9 dt_crit of the lumped system")
    states = {}
    for prec in ("fp32", "fp64"):
        ctx = fcw.assemble_cells(cfg, precision=prec)
        g = fcw.iga_create(ctx)
        info = fcw.iga_query(g)
        if prec == "fp32":
            dt = 0.9 * fcw.iga_critical_dt(g, max_iter=4000, rtol=1e-7)
        dtype = torch.float32 if prec == "fp32" else torch.float64
        u = torch.zeros((1, info["ndof"]), dtype=dtype, device="cuda:0")
        d = torch.zeros_like(u)
        fcw.iga_step(g, 1, u, d, src, 0.0, dt, warmup, 1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fcw.iga_step(g, 1, u, d, src, warmup * dt, dt, steps, 0)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        mass = fcw.iga_export(g, fcw.FCW_IGA_ARR_MASS)
        active = int((mass > 0).sum())
        states[prec] = u[0].double().cpu().numpy()
        ncut = info["n_cut"]
        fcw.iga_destroy(g)
        fcw.destroy(ctx)
        if prec == "fp32":
            ns = info["n_s"]
            ncells = 512 * 512
            byts = 5 * 4 * info["ndof"] + ncut * ns * ns * 4 + 4 * ncells
            flops = 2 * ns * ns * (info["n_cut"] + info["n_uncut"])
            t = ms * 1e-3 / steps
            hbm = dict(bound="hbm", achieved=byts / t / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                       frac=byts / t / 1e9 / HBM_PEAK_GBS, algorithmic_bytes_per_launch=byts)
            alu = dict(bound="alu", achieved=flops / t / 1e12, peak=157.3, unit="TFLOP/s",
                       frac=flops / t / 1e12 / 157.3, algorithmic_flops_per_launch=flops)
            main, other = (hbm, alu) if byts / (HBM_PEAK_GBS * 1e9) >= flops / 157.3e12 else (alu, hbm)
            main = dict(main, kernel="fcw::iga_step_kernel<float, 2, 4>", other=other,
                        note="ms_per_step includes the launch of each step (one kernel per step)")
            out.update(value=active * steps / (ms * 1e-3), unit="DOF-updates/s",
                       ms_per_step=ms / steps, steps=steps, ndof=info["ndof"], active_dof=active,
                       n_cut=ncut, dt=dt, dt_crit=info["dt_crit"] or dt / 0.9, roofline=main)
        else:
            out["fp64_ms_per_step"] = ms / steps
    out["rel_l2_fp32_vs_fp64"] = float(np.linalg.norm(states["fp32"] - states["fp64"])
                                       / np.linalg.norm(states["fp64"]))
    return out


def bench_serve(count, scale, rate, quantum):
    """Serving loop over the first `count` requests of the request stream (seed 5),
    cell counts per side scaled by `scale`; Poisson arrivals at `rate` requests/s
    (None: all at t=0)."""
    import workloads
    from paper_2501_19013_amd.serve import Server, requests_from_stream
    reqs = requests_from_stream(workloads.request_stream(seed=5, count=count, rate=rate),
                                scale=scale)
    srv = Server(precision="fp32", quantum=quantum)
    m = srv.run(reqs, log=lambda msg: print(f"[bench] serving {msg}", file=sys.stderr, flush=True))
    srv.close()
    n2 = sum(1 for r in reqs if r.cfg["dim"] == 2)
    m.update(requests=count, scale=scale, rate_per_s=rate, quantum=quantum,
             mix=f"{n2} 2-D, {count - n2} 3-D scalar; p in 2-4; 200-2000 steps",
             workload=f"first {count} requests of the serving stream (seed 5), cell counts per "
                      f"side x{scale:g}, FP32 step, FP64 setup per request, arrivals "
                      + ("all at t=0" if rate is None else f"Poisson {rate:g}/s"))
    print(f"[bench] serving: {m['n']} requests in {m['makespan_s']:.1f} s, p50 "
          f"{m['p50_latency_s']:.2f} s, p99 {m['p99_latency_s']:.2f} s", file=sys.stderr, flush=True)
    return m


def calibrate_copy(nbytes=1 << 30):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1800)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=200,
                    help="oracle steps on all host threads (also the parity check's length)")
    ap.add_argument("--cpu-steps-1t", type=int, default=40, help="oracle steps on one thread")
    ap.add_argument("--calib", action="store_true", help="also run a 1 GiB copy (counter scale)")
    ap.add_argument("--no-c3", action="store_true", help="skip the 3-D elastic workload")
    ap.add_argument("--imex-steps", type=int, default=200,
                    help="steps of the IMEX leg (0 skips it)")
    ap.add_argument("--imex-full-steps", type=int, default=100,
                    help="steps of the IMEX leg at the full c2 size (0 skips it)")
    ap.add_argument("--iga-steps", type=int, default=500, help="steps of the IGA-FCM leg (0: skip)")
    ap.add_argument("--c3-steps", type=int, default=1000)
    ap.add_argument("--c4-steps", type=int, default=0,
                    help="steps of the 3-D elastic p=3 leg with 16 right-hand sides (0: skip)")
    ap.add_argument("--c3-warmup", type=int, default=10)
    ap.add_argument("--serve-count", type=int, default=64, help="requests of the serving leg (0: skip)")
    ap.add_argument("--serve-scale", type=float, default=0.5, help="cell counts per side x this")
    ap.add_argument("--serve-rate", type=float, default=2.0, help="Poisson arrivals per s (<=0: all at 0)")
    ap.add_argument("--serve-quantum", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "domain decomposition is a design, not a build, in this repository",
              file=sys.stderr)
        sys.exit(2)

    import workloads
    cfg = workloads.config("c2")
    r32 = run_gpu(cfg, "fp32", args.steps, args.warmup)
    print(f"[bench] fp32: {args.steps} steps in {r32['ms']:.2f} ms", file=sys.stderr, flush=True)
    res = dict(metric="DOF-updates/s at \u22641e-4 rel L2 vs FP64 oracle (FP32 vs FP64); p99 latency",
               unit="DOF-updates/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic")
    ms_step = r32["ms"] / args.steps
    res["value"] = r32["active"] * args.steps / (r32["ms"] * 1e-3)
    res["ms_per_step"] = ms_step
    info = r32["info"]
    res["roofline"] = roofline(cfg, r32, "fp32")
    res["config"] = dict(workload="c2: 2-D scalar wave, [0,1]^2, 40 random circular voids "
                                  "(r 0.01-0.05, seed 2), 512x512 cells, p=4 GLL, FP32 step, "
                                  "FP64 setup, Ricker f0=10 at (0.1,0.1), dt=0.9 dt_crit",
                         ndof=info["ndof"], active_dof=r32["active"], n_cut=info["n_cut"],
                         n_uncut=info["n_uncut"], n_out=info["n_out"], dt=r32["dt"],
                         dt_crit=info["dt_crit"], total_steps=args.warmup + args.steps)
    if not args.no_fp64:
        r64 = run_gpu(cfg, "fp64", args.steps, args.warmup, dt=r32["dt"])
        print(f"[bench] fp64: {args.steps} steps in {r64['ms']:.2f} ms", file=sys.stderr, flush=True)
        e = float(np.linalg.norm(r32["u"] - r64["u"]) / np.linalg.norm(r64["u"]))
        v64 = r64["active"] * args.steps / (r64["ms"] * 1e-3)
        res["fp64_gpu"] = dict(value=v64, ms_per_step=r64["ms"] / args.steps)
        res["speedup_vs_fp64_gpu"] = res["value"] / v64
        res["rel_l2_vs_fp64"] = e
    res["p99_latency_s"] = None
    if not args.no_cpu:
        cb, dt_orc, ref = cpu_baseline(cfg, args.cpu_steps, args.cpu_steps_1t)
        res["cpu_baseline"] = cb
        print(f"[bench] cpu baseline: {cb['sample']}", file=sys.stderr, flush=True)
        # parity of the timed forms against the oracle's state, same steps from rest
        nref = float(np.linalg.norm(ref))
        par = dict(steps=args.cpu_steps, dt=dt_orc, tolerance=1e-4,
                   full_length="2000 steps: tests/test_gpu_c2_full_length.py")
        for prec in ("fp32", "fp64"):
            par[prec] = float(np.linalg.norm(gpu_state(cfg, prec, dt_orc, args.cpu_steps) - ref)
                              / nref)
        res["rel_l2_vs_oracle"] = par
        if par["fp32"] > 1e-4:
            res["value_flag"] = "FP32 state above the 1e-4 tolerance against the oracle"
        print(f"[bench] rel L2 vs oracle after {args.cpu_steps} steps: fp32 {par['fp32']:.2e}, "
              f"fp64 {par['fp64']:.2e}", file=sys.stderr, flush=True)
    if not args.no_c3:
        res["c3"] = bench_c3(args.c3_steps, args.c3_warmup, not args.no_fp64)
    if args.c4_steps > 0:
        res["c4"] = bench_c4(args.c4_steps, 2)
        print(f"[bench] c4: {res['c4']['ms_per_step']:.2f} ms/step for 16 right-hand sides",
              file=sys.stderr, flush=True)
    if args.imex_steps > 0:
        res["imex"] = bench_imex(args.imex_steps, 5, args.imex_full_steps)
        print(f"[bench] imex: {res['imex']['ms_per_step']:.3f} ms/step, "
              f"{res['imex']['n_implicit']} implicit DOFs in {res['imex']['n_blocks']} blocks",
              file=sys.stderr, flush=True)
        if "c2_full" in res["imex"]:
            f = res["imex"]["c2_full"]
            print(f"[bench] imex c2 full size: {f['ms_per_step']:.3f} ms/step, "
                  f"{f['n_implicit']} implicit DOFs in {f['n_blocks']} blocks (largest "
                  f"{f['largest_block']}), set-up {f['prepare_s']:.1f} s, explicit "
                  f"{f['explicit_ms_per_step']:.3f} ms/step, {f['batch_rhs']} right-hand sides "
                  f"{f['batch_ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if args.iga_steps > 0:
        res["iga"] = bench_iga(args.iga_steps, 10)
        print(f"[bench] iga: {res['iga']['ms_per_step'] * 1e3:.1f} us/step", file=sys.stderr,
              flush=True)
    if args.serve_count > 0:
        res["serving"] = bench_serve(args.serve_count, args.serve_scale,
                                     None if args.serve_rate <= 0 else args.serve_rate,
                                     args.serve_quantum)
        res["p99_latency_s"] = res["serving"]["p99_latency_s"]
    if args.calib:
        calibrate_copy()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
