"""ctypes binding of the fcw C ABI (include/fcw.h).

Argument marshalling only: every computation runs in the HIP kernels of libfcw.so.
Device buffers are passed as raw pointers; anything with a ``data_ptr()`` method
(a torch tensor on the GPU) is accepted as well.  Loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfcw.so")

FCW_OK, FCW_E_ARG, FCW_E_NOMEM, FCW_E_DEVICE, FCW_E_STATE, FCW_E_NOCONV, FCW_E_UNSTABLE, \
    FCW_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
FCW_FP64, FCW_FP32, FCW_BF16 = 0, 1, 2
PRECISIONS = {"fp64": FCW_FP64, "fp32": FCW_FP32, "bf16": FCW_BF16}
(ARR_CELL_CLASS, ARR_CUT_CELLS, ARR_K_REF, ARR_K_CUT, ARR_M_CUT, ARR_LUMPED_CUT, ARR_MASS,
 ARR_EVS_MARGIN, ARR_IMEX_DOFS) = range(9)
_ARR_DTYPE = {ARR_CELL_CLASS: np.int8, ARR_CUT_CELLS: np.int32, ARR_IMEX_DOFS: np.int64}

# every entry point declared in include/fcw.h
EXPORTS = ("fcw_assemble_cells", "fcw_stabilize_cut_cells", "fcw_critical_dt",
           "fcw_step_explicit", "fcw_step_explicit_noalloc", "fcw_imex_prepare", "fcw_imex_layout", "fcw_step_imex", "fcw_step_consistent",
           "fcw_apply_stiffness",
           "fcw_query",
           "fcw_autotune", "fcw_tile_config", "fcw_tile_name", "fcw_select_tile", "fcw_set_stream", "fcw_kernel_times", "fcw_run",
           "fcw_export", "fcw_destroy", "fcw_last_error", "fcw_trace_error",
           "fcw_iga_create", "fcw_iga_critical_dt", "fcw_iga_step", "fcw_iga_apply_stiffness",
           "fcw_iga_query", "fcw_iga_export", "fcw_iga_destroy")


class ProblemDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("ncomp", C.c_int32), ("ncells", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("p", C.c_int32),
                ("tree_depth", C.c_int32), ("nvoids", C.c_int32),
                ("void_center", C.POINTER(C.c_double)), ("void_radius", C.POINTER(C.c_double)),
                ("alpha", C.c_double), ("rho", C.c_double), ("c", C.c_double), ("E", C.c_double),
                ("nu", C.c_double), ("precision", C.c_int32), ("stream", C.c_void_p),
                ("cube_center", C.c_double * 3), ("cube_half", C.c_double),
                ("cube_rot", C.c_double * 9)]


class Source(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("dir", C.c_double * 3), ("f0", C.c_double),
                ("amp", C.c_double), ("sigma", C.c_double)]


class RunResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps_done", C.c_int32), ("dt_used", C.c_double),
                ("growth", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RunItem(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("nrhs", C.c_int32), ("u", C.c_void_p), ("d", C.c_void_p),
                ("src", C.POINTER(Source)), ("t0", C.c_double), ("dt", C.c_double),
                ("dt_max", C.c_double), ("nsteps", C.c_int32), ("start", C.c_int32),
                ("nrec", C.c_int32), ("rec_x", C.POINTER(C.c_double)),
                ("traces", C.c_void_p), ("check_every", C.c_int32),
                ("result", C.POINTER(RunResult)), ("energy", C.POINTER(C.c_double))]


MAX_RECEIVERS = 64


FCW_RUN_GRAPH = 1


class Info(C.Structure):
    _fields_ = [("ndof", C.c_int64), ("nnodes", C.c_int64), ("ncells", C.c_int64),
                ("n_cut", C.c_int64), ("n_uncut", C.c_int64), ("n_out", C.c_int64),
                ("n_loc", C.c_int32), ("precision", C.c_int32), ("footprint_bytes", C.c_int64),
                ("dt_crit", C.c_double), ("min_evs_margin", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IgaInfo(C.Structure):
    _fields_ = [("ndof", C.c_int64), ("nbasis", C.c_int32 * 3), ("n_s", C.c_int32),
                ("precision", C.c_int32), ("n_cut", C.c_int64), ("n_uncut", C.c_int64),
                ("n_out", C.c_int64), ("dt_crit", C.c_double), ("footprint_bytes", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["nbasis"] = tuple(self.nbasis)
        return d


FCW_IGA_ARR_MASS, FCW_IGA_ARR_K_CLASS, FCW_IGA_ARR_K_CUT = 0, 1, 2


class FcwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fcw status {status}: {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load libfcw.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_2501_19013_amd/build.py")
    lib = C.CDLL(path)
    vp, i32, f64 = C.c_void_p, C.c_int32, C.c_double
    lib.fcw_assemble_cells.argtypes = [C.POINTER(ProblemDesc), C.POINTER(vp)]
    lib.fcw_stabilize_cut_cells.argtypes = [vp, f64, f64]
    lib.fcw_critical_dt.argtypes = [vp, i32, f64, C.POINTER(f64)]
    lib.fcw_step_explicit.argtypes = [vp, i32, vp, vp, C.POINTER(Source), f64, f64, i32, i32]
    lib.fcw_step_explicit_noalloc.argtypes = [vp, i32, vp, vp, C.POINTER(Source), f64, f64, i32,
                                              i32]
    lib.fcw_imex_prepare.argtypes = [vp, f64, C.POINTER(C.c_int64)]
    lib.fcw_imex_layout.argtypes = [vp, C.POINTER(i32), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]
    lib.fcw_step_imex.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(Source), f64, f64, i32, i32]
    lib.fcw_step_consistent.argtypes = [vp, i32, vp, vp, C.POINTER(Source), f64, f64, i32, i32]
    lib.fcw_apply_stiffness.argtypes = [vp, i32, vp, vp]
    lib.fcw_query.argtypes = [vp, C.POINTER(Info)]
    lib.fcw_export.argtypes = [vp, i32, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.fcw_autotune.argtypes = [vp, i32, i32, C.POINTER(i32)]
    lib.fcw_tile_config.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(f64), C.POINTER(i32)]
    lib.fcw_select_tile.argtypes = [vp, i32]
    lib.fcw_tile_name.argtypes = [vp, i32, C.c_char_p, i32]
    lib.fcw_set_stream.argtypes = [vp, vp]
    lib.fcw_kernel_times.argtypes = [vp, i32, i32, C.POINTER(f64), C.POINTER(f64)]
    lib.fcw_run.argtypes = [C.POINTER(RunItem), i32, i32]
    lib.fcw_trace_error.argtypes = [C.POINTER(f64), C.c_int64, C.POINTER(f64), C.c_int64, i32,
                                    i32, C.POINTER(f64)]
    lib.fcw_destroy.argtypes = [vp]
    lib.fcw_destroy.restype = None
    lib.fcw_last_error.argtypes = []
    lib.fcw_last_error.restype = C.c_char_p
    lib.fcw_iga_create.argtypes = [vp, C.POINTER(vp)]
    lib.fcw_iga_critical_dt.argtypes = [vp, i32, f64, C.POINTER(f64)]
    lib.fcw_iga_step.argtypes = [vp, i32, vp, vp, C.POINTER(Source), f64, f64, i32, i32]
    lib.fcw_iga_apply_stiffness.argtypes = [vp, i32, vp, vp]
    lib.fcw_iga_query.argtypes = [vp, C.POINTER(IgaInfo)]
    lib.fcw_iga_export.argtypes = [vp, i32, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.fcw_iga_destroy.argtypes = [vp]
    lib.fcw_iga_destroy.restype = None
    for name in EXPORTS:
        if name not in ("fcw_destroy", "fcw_last_error", "fcw_iga_destroy"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(status):
    if status != FCW_OK:
        raise FcwError(status, load().fcw_last_error().decode())
    return status


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _sources(srcs):
    if not srcs:
        return None
    arr = (Source * len(srcs))()
    for i, s in enumerate(srcs):
        x = tuple(s["x"]) + (0.0,) * (3 - len(s["x"]))
        d = tuple(s.get("dir", (1.0, 0.0, 0.0)))
        d = d + (0.0,) * (3 - len(d))
        arr[i].x[:] = x
        arr[i].dir[:] = d[:3]
        arr[i].f0 = float(s.get("f0", 10.0))
        arr[i].amp = float(s.get("amp", 1.0))
        arr[i].sigma = float(s.get("sigma", 0.0))
    return arr


def assemble_cells(cfg, precision="fp64", stream=None):
    """fcw_assemble_cells from a configuration dict (keys as in ``workloads``)."""
    lib = load()
    dim = int(cfg["dim"])
    desc = ProblemDesc()
    desc.dim = dim
    desc.ncomp = int(cfg.get("ncomp", 1))
    nc = list(cfg["ncells"]) + [1] * (3 - dim)
    desc.ncells[:] = [int(v) for v in nc]
    desc.lo[:] = list(cfg["lo"]) + [0.0] * (3 - dim)
    desc.hi[:] = list(cfg["hi"]) + [0.0] * (3 - dim)
    desc.p = int(cfg["p"])
    desc.tree_depth = int(cfg.get("tree_depth", 3))
    vc = np.ascontiguousarray(cfg["void_center"], dtype=np.float64).reshape(-1)
    vr = np.ascontiguousarray(cfg["void_radius"], dtype=np.float64).reshape(-1)
    desc.nvoids = len(vr)
    desc.void_center = vc.ctypes.data_as(C.POINTER(C.c_double))
    desc.void_radius = vr.ctypes.data_as(C.POINTER(C.c_double))
    desc.alpha = float(cfg.get("alpha", 1e-12))
    desc.rho = float(cfg.get("rho", 1.0))
    desc.c = float(cfg.get("c", 1.0))
    desc.E = float(cfg.get("E", 1.0))
    desc.nu = float(cfg.get("nu", 0.3))
    desc.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    desc.stream = stream
    cube = cfg.get("cube")
    if cube is not None:
        desc.cube_center[:] = [float(v) for v in list(cube["center"]) + [0.0] * (3 - dim)]
        desc.cube_half = float(cube["half"])
        rot = np.zeros((3, 3))
        rot[:dim, :dim] = np.asarray(cube["rot"], dtype=np.float64).reshape(dim, dim)
        desc.cube_rot[:] = [float(v) for v in rot.ravel()]
    ctx = C.c_void_p()
    _check(lib.fcw_assemble_cells(C.byref(desc), C.byref(ctx)))
    return ctx


def stabilize_cut_cells(ctx, eps, f_lambda):
    _check(load().fcw_stabilize_cut_cells(ctx, float(eps), float(f_lambda)))


def critical_dt(ctx, max_iter=4000, rtol=1e-9):
    out = C.c_double()
    _check(load().fcw_critical_dt(ctx, int(max_iter), float(rtol), C.byref(out)))
    return out.value


def step_explicit(ctx, nrhs, u, d, sources, t0, dt, nsteps, start):
    srcs = _sources(sources)
    _check(load().fcw_step_explicit(ctx, int(nrhs), _ptr(u), _ptr(d), srcs, float(t0),
                                    float(dt), int(nsteps), int(start)))


def step_explicit_noalloc(ctx, nrhs, u, d, sources, t0, dt, nsteps, start):
    """fcw_step_explicit_noalloc: the explicit step with its work areas in the library's
    fixed per-device array (no device allocation during the call)."""
    srcs = _sources(sources)
    _check(load().fcw_step_explicit_noalloc(ctx, int(nrhs), _ptr(u), _ptr(d), srcs, float(t0),
                                            float(dt), int(nsteps), int(start)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def imex_prepare(ctx, dt):
    """Number of implicit DOFs of the IMEX scheme for step size dt (sets it up)."""
    n = C.c_int64()
    _check(load().fcw_imex_prepare(ctx, float(dt), C.byref(n)))
    return n.value


def imex_layout(ctx):
    """Blocks of the prepared implicit set: dict(n_blocks, largest, solve_bytes)."""
    nb, lg, sb = C.c_int32(), C.c_int64(), C.c_int64()
    _check(load().fcw_imex_layout(ctx, C.byref(nb), C.byref(lg), C.byref(sb)))
    return dict(n_blocks=nb.value, largest=lg.value, solve_bytes=sb.value)


def step_consistent(ctx, nrhs, u, d, sources, t0, dt, nsteps, start):
    srcs = _sources(sources)
    _check(load().fcw_step_consistent(ctx, int(nrhs), _ptr(u), _ptr(d), srcs, float(t0),
                                      float(dt), int(nsteps), int(start)))


def step_imex(ctx, nrhs, u, d, v_c, a_c, sources, t0, dt, nsteps, start):
    srcs = _sources(sources)
    _check(load().fcw_step_imex(ctx, int(nrhs), _ptr(u), _ptr(d), _ptr(v_c), _ptr(a_c), srcs,
                                float(t0), float(dt), int(nsteps), int(start)))


def apply_stiffness(ctx, nrhs, u, r):
    _check(load().fcw_apply_stiffness(ctx, int(nrhs), _ptr(u), _ptr(r)))


def autotune(ctx, nrhs=1, nsteps=20):
    """Time every tile configuration and keep the fastest; returns (chosen, table)."""
    lib = load()
    ch = C.c_int32()
    _check(lib.fcw_autotune(ctx, int(nrhs), int(nsteps), C.byref(ch)))
    return ch.value, tile_configs(ctx)


def tile_configs(ctx):
    lib = load()
    n = C.c_int32()
    lib.fcw_tile_config(ctx, 0, None, None, C.byref(n))
    out = []
    for i in range(n.value):
        t = (C.c_int32 * 3)()
        us = C.c_double()
        _check(lib.fcw_tile_config(ctx, i, t, C.byref(us), None))
        name = C.create_string_buffer(256)
        _check(lib.fcw_tile_name(ctx, i, name, 256))
        out.append(dict(tile=tuple(t), us_per_step=us.value, kernel=name.value.decode()))
    return out


def run(entries, graph=False, raise_unstable=True):
    """fcw_run.  Each entry is a dict with ctx, nrhs, u, d and optionally sources, t0, dt
    (<= 0: the library's rule min(0.9 dt_crit, dt_max)), dt_max, nsteps, start,
    receivers ([nrec][dim] points), traces (device double [nrhs][nsteps+1][nrec][ncomp]),
    check_every, energy (True: return the discrete energy per right-hand side).
    Returns one dict per entry: status, steps_done, dt_used, growth (and energy)."""
    arr = (RunItem * len(entries))()
    keep, results, energies = [], [], []
    for i, e in enumerate(entries):
        srcs = _sources(e.get("sources"))
        keep.append(srcs)
        arr[i].ctx = e["ctx"].value if isinstance(e["ctx"], C.c_void_p) else e["ctx"]
        arr[i].nrhs = int(e["nrhs"])
        arr[i].u = _ptr(e["u"])
        arr[i].d = _ptr(e["d"])
        arr[i].src = C.cast(srcs, C.POINTER(Source)) if srcs is not None else None
        arr[i].t0 = float(e.get("t0", 0.0))
        arr[i].dt = float(e.get("dt", 0.0))
        arr[i].dt_max = float(e.get("dt_max", 0.0))
        arr[i].nsteps = int(e["nsteps"])
        arr[i].start = int(e.get("start", 0))
        rec = e.get("receivers")
        if rec is not None and len(rec):
            pts = np.zeros((len(rec), 3))
            for q, x in enumerate(rec):
                pts[q, :len(x)] = x
            pts = np.ascontiguousarray(pts)
            keep.append(pts)
            arr[i].nrec = len(rec)
            arr[i].rec_x = pts.ctypes.data_as(C.POINTER(C.c_double))
            arr[i].traces = _ptr(e["traces"])
        arr[i].check_every = int(e.get("check_every", 0))
        res = RunResult()
        results.append(res)
        arr[i].result = C.pointer(res)
        en = None
        if e.get("energy"):
            en = (C.c_double * int(e["nrhs"]))()
            arr[i].energy = C.cast(en, C.POINTER(C.c_double))
        energies.append(en)
    status = load().fcw_run(arr, len(entries), FCW_RUN_GRAPH if graph else 0)
    if status != FCW_OK and not (status == FCW_E_UNSTABLE and not raise_unstable):
        _check(status)
    out = []
    for res, en in zip(results, energies):
        d = res.as_dict()
        if en is not None:
            d["energy"] = list(en)
        out.append(d)
    return out


def select_tile(ctx, i):
    _check(load().fcw_select_tile(ctx, int(i)))


def set_stream(ctx, stream):
    """fcw_set_stream: later work of ``ctx`` goes on ``stream`` (a hipStream_t handle)."""
    _check(load().fcw_set_stream(ctx, stream))


def kernel_times(ctx, nrhs=1, nsteps=100):
    """fcw_kernel_times: (main kernel, cut-cell kernel) microseconds per launch."""
    m, c = C.c_double(), C.c_double()
    _check(load().fcw_kernel_times(ctx, int(nrhs), int(nsteps), C.byref(m), C.byref(c)))
    return m.value, c.value


def query(ctx):
    info = Info()
    _check(load().fcw_query(ctx, C.byref(info)))
    return info.as_dict()


def export(ctx, which):
    lib = load()
    n = C.c_int64()
    _check(lib.fcw_export(ctx, int(which), None, 0, C.byref(n)))
    out = np.empty(n.value, dtype=_ARR_DTYPE.get(which, np.float64))
    _check(lib.fcw_export(ctx, int(which), out.ctypes.data, n.value, C.byref(n)))
    return out


def trace_error(sim, ref, sim_stride, ref_stride, n_samples):
    """fcw_trace_error: eq. error of host traces [rows][n_obs] sampled every sim_stride /
    ref_stride rows (rows 1 .. n_samples of each)."""
    sim = np.ascontiguousarray(sim, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    nobs = sim.shape[1]
    if (ref.shape[1] != nobs or sim.shape[0] < n_samples * sim_stride + 1
            or ref.shape[0] < n_samples * ref_stride + 1):
        raise ValueError("traces too short for the requested samples")
    e = C.c_double()
    P = C.POINTER(C.c_double)
    _check(load().fcw_trace_error(sim.ctypes.data_as(P), int(sim_stride), ref.ctypes.data_as(P),
                                  int(ref_stride), int(n_samples), int(nobs), C.byref(e)))
    return e.value


def destroy(ctx):
    if ctx:
        load().fcw_destroy(ctx)


def iga_create(ctx):
    """fcw_iga_create: the B-spline (IGA-FCM) problem on the assembled cells of ``ctx``."""
    g = C.c_void_p()
    _check(load().fcw_iga_create(ctx, C.byref(g)))
    return g


def iga_critical_dt(g, max_iter=4000, rtol=1e-9):
    out = C.c_double()
    _check(load().fcw_iga_critical_dt(g, int(max_iter), float(rtol), C.byref(out)))
    return out.value


def iga_step(g, nrhs, u, d, sources, t0, dt, nsteps, start):
    srcs = _sources(sources)
    _check(load().fcw_iga_step(g, int(nrhs), _ptr(u), _ptr(d), srcs, float(t0), float(dt),
                               int(nsteps), int(start)))


def iga_apply_stiffness(g, nrhs, u, r):
    _check(load().fcw_iga_apply_stiffness(g, int(nrhs), _ptr(u), _ptr(r)))


def iga_query(g):
    info = IgaInfo()
    _check(load().fcw_iga_query(g, C.byref(info)))
    return info.as_dict()


def iga_export(g, which):
    lib = load()
    n = C.c_int64()
    _check(lib.fcw_iga_export(g, int(which), None, 0, C.byref(n)))
    out = np.empty(n.value, dtype=np.float64)
    _check(lib.fcw_iga_export(g, int(which), out.ctypes.data, n.value, C.byref(n)))
    return out


def iga_destroy(g):
    if g:
        load().fcw_iga_destroy(g)


def last_error():
    return load().fcw_last_error().decode()
