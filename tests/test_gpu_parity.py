"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: the FP64 path computes the same finite recurrence as the oracle with a
different summation order, so its relative L2 error stays at a few hundred ulps
(1e-10 is the bar); the FP32 path is held to 1e-4 relative L2 (the bar of the FP32
form), measured over the active DOFs at every checkpoint.  Integer results (cell
classes, cut-cell lists) are compared bit for bit.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import geometry, problem, timestep

pytestmark = pytest.mark.gpu


def _solver(cfg, precision):
    from paper_2501_19013_amd.solver import Solver
    return Solver(cfg, precision=precision)


def _oracle(cfg):
    return problem.build(problem.Problem.from_config(cfg))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c1():
    cfg = workloads.config("c1")
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    return cfg, disc, dt


def _setup_parity(cfg, disc, s):
    from paper_2501_19013_amd import fcw
    cls = s.export(fcw.ARR_CELL_CLASS)
    np.testing.assert_array_equal(cls, disc.cls)
    cand = s.export(fcw.ARR_CUT_CELLS)
    kept = cand[cls[cand] == geometry.CUT]
    np.testing.assert_array_equal(kept, disc.cut_cells)
    nl, ns = disc.prob.n_loc, disc.prob.n_s
    kref = s.export(fcw.ARR_K_REF).reshape(nl, nl)
    np.testing.assert_allclose(kref, disc.K_ref, atol=1e-13 * np.abs(disc.K_ref).max())
    keep = cls[cand] == geometry.CUT
    kc = s.export(fcw.ARR_K_CUT).reshape(-1, nl, nl)[keep]
    mc = s.export(fcw.ARR_M_CUT).reshape(-1, ns, ns)[keep]
    lc = s.export(fcw.ARR_LUMPED_CUT).reshape(-1, ns)[keep]
    for q in range(len(kept)):
        sc = np.abs(disc.K_cut[q]).max()
        assert np.abs(kc[q] - disc.K_cut[q]).max() <= 1e-12 * sc, q
        assert np.abs(mc[q] - disc.Mo_cut[q]).max() <= 1e-13 * np.abs(disc.Mo_cut[q]).max(), q
        assert np.abs(lc[q] - disc.lumped_cut[q]).max() <= 1e-10 * np.abs(disc.lumped_cut[q]).max(), q
    mass = s.export(fcw.ARR_MASS)
    np.testing.assert_allclose(mass, disc.mass, rtol=1e-10, atol=1e-14 * disc.mass.max())


def test_c1_setup_parity(c1):
    cfg, disc, _ = c1
    s = _solver(cfg, "fp64")
    _setup_parity(cfg, disc, s)
    info = s.info
    assert info["n_cut"] == len(disc.cut_cells) == 28
    assert info["n_out"] == 32 and info["n_uncut"] == 196
    # the eigenvalue split is decided far from rounding in every cut cell
    assert info["min_evs_margin"] > 1e-10
    assert abs(info["min_evs_margin"] - disc.evs_margin.min()) < 1e-8
    s.close()


def test_c1_critical_dt(c1):
    cfg, disc, _ = c1
    s = _solver(cfg, "fp64")
    dtc = s.critical_dt(max_iter=2000, rtol=1e-13)
    ref = timestep.critical_dt(disc)
    assert abs(dtc - ref) <= 1e-8 * ref
    s.close()


def test_critical_dt_midsize():
    # 128^2 cells p=4 (263k nodes) of the 2-D void field: the device Lanczos stops on the
    # residual of its Ritz pair and reports theta + residual, which lies within rtol of
    # the oracle's lambda_max and not below it
    cfg = workloads.scaled_config(2, 128, 4, seed=2)
    disc = problem.build(problem.Problem.from_config(cfg))
    ref = timestep.critical_dt(disc)
    s = _solver(cfg, "fp64")
    dtc = s.critical_dt(max_iter=4000, rtol=1e-9)
    s.close()
    assert abs(dtc - ref) <= 1e-8 * ref
    assert dtc <= ref * (1.0 + 1e-11)


def test_critical_dt_reports_nonconvergence(c1):
    # an iteration cap too small for the tolerance is an error, not a silent estimate
    from paper_2501_19013_amd import fcw
    cfg, _, _ = c1
    s = _solver(cfg, "fp64")
    with pytest.raises(fcw.FcwError) as e:
        fcw.critical_dt(s.ctx, 20, 1e-15)
    assert e.value.status == fcw.FCW_E_NOCONV
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_stiffness_action(c1, precision):
    import torch
    cfg, disc, _ = c1
    s = _solver(cfg, precision)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((2, disc.prob.ndof)) * (disc.mass > 0)
    ug = torch.tensor(u, dtype=s.dtype, device="cuda")
    r = s.apply_stiffness(ug).double().cpu().numpy()
    for k in range(2):
        ref = problem.apply_K(disc, u[k])
        tol = 1e-13 if precision == "fp64" else 2e-6
        assert np.abs(r[k] - ref).max() <= tol * np.abs(ref).max()
    s.close()


def _run_gpu(s, cfg, dt, nsteps, chunks):
    """Run in chunks (t0 advances), returning u after each chunk end."""
    import torch
    u = s.zeros(1)
    d = s.zeros(1)
    out = {}
    k = 0
    for n in chunks:
        s.step(u, d, cfg["sources"], dt, n, t0=k * dt, start=(k == 0))
        k += n
        torch.cuda.synchronize()
        out[k] = u[0].double().cpu().numpy().copy()
    assert k == nsteps
    return out


def test_c1_fp64_run_parity(c1):
    cfg, disc, dt = c1
    s = _solver(cfg, "fp64")
    chunks = [1, 99, 100, 101, 199]   # odd and even chunk lengths, the start step alone
    got = _run_gpu(s, cfg, dt, 500, chunks)
    ref = timestep.cdm(disc, dt, 500, sources=cfg["sources"], checkpoints=tuple(got))
    for k, u in got.items():
        e = rel_l2(u, ref["snapshots"][k])
        assert e <= 1e-10, (k, e)
    s.close()


def test_c1_fp32_run_parity(c1):
    cfg, disc, dt = c1
    s = _solver(cfg, "fp32")
    got = _run_gpu(s, cfg, dt, 500, [100] * 5)
    ref = timestep.cdm(disc, dt, 500, sources=cfg["sources"], checkpoints=tuple(got))
    for k, u in got.items():
        e = rel_l2(u, ref["snapshots"][k])
        assert e <= 1e-4, (k, e)
    s.close()


@pytest.fixture(scope="module")
def c2_small():
    # the c2 void field (seed 2, 40 circles, r in [0.01, 0.05]) on 64x64 cells, p = 4:
    # several tiles in each direction and a ragged tail in neither; 400 steps
    cfg = workloads.config("c2")
    cfg["ncells"] = (64, 64)
    cfg["nsteps"] = 400
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    return cfg, disc, dt


def test_c2_small_setup_parity(c2_small):
    cfg, disc, _ = c2_small
    s = _solver(cfg, "fp64")
    _setup_parity(cfg, disc, s)
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_c2_small_run_parity(c2_small, precision, tol):
    cfg, disc, dt = c2_small
    s = _solver(cfg, precision)
    got = _run_gpu(s, cfg, dt, 400, [200, 200])
    ref = timestep.cdm(disc, dt, 400, sources=cfg["sources"], checkpoints=tuple(got))
    for k, u in got.items():
        e = rel_l2(u, ref["snapshots"][k])
        assert e <= tol, (k, e)
    s.close()


def test_ragged_grid_and_multi_rhs():
    # non-square grid whose sizes are not multiples of any tile edge, three sources
    # as three right-hand sides; each must equal its own oracle run
    import torch
    cfg = workloads.config("c2")
    h = 1.0 / 48
    cfg.update(ncells=(37, 23), hi=(37 * h, 23 * h), p=3, nsteps=150)
    cc, rr = workloads.random_circles(seed=12, count=8, rmin=0.03, rmax=0.08,
                                      hi=23 * h, keep_clear=((0.1, 0.1), (0.6, 0.3), (0.3, 0.4)))
    cfg["void_center"], cfg["void_radius"] = cc, rr
    srcs = [dict(x=(0.1, 0.1), f0=10.0, amp=1.0), dict(x=(0.6, 0.3), f0=12.0, amp=0.5),
            dict(x=(0.3, 0.4), f0=8.0, amp=2.0)]
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    for precision, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        s = _solver(cfg, precision)
        _setup_parity(cfg, disc, s) if precision == "fp64" else None
        u = s.zeros(3)
        d = s.zeros(3)
        s.step(u, d, srcs, dt, 150, t0=0.0, start=True)
        torch.cuda.synchronize()
        ug = u.double().cpu().numpy()
        for r, src in enumerate(srcs):
            ref = timestep.cdm(disc, dt, 150, sources=[src])["u"]
            assert rel_l2(ug[r], ref) <= tol, (precision, r)
        s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_elastic_3d_parity(precision, tol):
    # 4^3 cells of the c3 pore-field kind (radii 0.02-0.06), octree depth 3
    cfg = workloads.scaled_config(3, 4, 2, seed=4, ncomp=3, porosity=0.2, nsteps=120)
    cfg["sources"] = [dict(x=(0.1, 0.1, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)]
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    s = _solver(cfg, precision)
    if precision == "fp64":
        _setup_parity(cfg, disc, s)
    got = _run_gpu(s, cfg, dt, 120, [60, 60])
    ref = timestep.cdm(disc, dt, 120, sources=cfg["sources"], checkpoints=tuple(got))
    for k, u in got.items():
        assert rel_l2(u, ref["snapshots"][k]) <= tol, k
    s.close()


def test_scalar_3d_parity():
    cfg = workloads.scaled_config(3, 6, 3, seed=4, porosity=0.15, nsteps=80, depth=2)
    cfg["sources"] = [dict(x=(0.1, 0.1, 0.1), f0=10.0, amp=1.0)]
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    s = _solver(cfg, "fp64")
    _setup_parity(cfg, disc, s)
    got = _run_gpu(s, cfg, dt, 80, [80])
    ref = timestep.cdm(disc, dt, 80, sources=cfg["sources"])["u"]
    assert rel_l2(got[80], ref) <= 1e-10
    s.close()


def test_scalar_3d_p4_large_cell_stabilisation():
    # n_s = 125: the tridiagonal (Householder + QL) path of the stabilisation; cut cells
    # of a 6^3 pore field checked one by one against the oracle (cells with 0, 1 and 3
    # small eigenvalues; margins 1e-5 .. 1e-4)
    from paper_2501_19013_amd import fcw
    cfg = workloads.scaled_config(3, 6, 4, seed=6, porosity=0.2, nsteps=40, depth=2)
    cells = [98, 171, 206, 1, 95, 128]
    disc = problem.build(problem.Problem.from_config(cfg), cut_subset=cells)
    assert sorted(set(disc.evs_nsmall.tolist())) == [0, 1, 3]
    s = _solver(cfg, "fp64")
    cand = s.export(fcw.ARR_CUT_CELLS)
    lc = s.export(fcw.ARR_LUMPED_CUT).reshape(-1, 125)
    mc = s.export(fcw.ARR_M_CUT).reshape(-1, 125, 125)
    slot = {int(c): q for q, c in enumerate(cand)}
    for k, cell in enumerate(disc.cut_cells):
        q = slot[int(cell)]
        ref = disc.lumped_cut[k]
        assert np.abs(mc[q] - disc.Mo_cut[k]).max() <= 1e-13 * np.abs(disc.Mo_cut[k]).max()
        assert np.abs(lc[q] - ref).max() <= 1e-10 * np.abs(ref).max(), int(cell)
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_scalar_3d_p4_run_parity(precision, tol):
    # 3^3 cells, p=4, one offset ball (24 cut cells, one with 112 small eigenvalues),
    # octree depth 1
    cfg = workloads._base(3, (3, 3, 3), 4, [(0.55, 0.5, 0.45)], [0.3], tree_depth=1,
                          nsteps=60)
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    s = _solver(cfg, precision)
    if precision == "fp64":
        _setup_parity(cfg, disc, s)
    got = _run_gpu(s, cfg, dt, 60, [25, 35])
    ref = timestep.cdm(disc, dt, 60, sources=cfg["sources"], checkpoints=tuple(got))
    for k, u in got.items():
        assert rel_l2(u, ref["snapshots"][k]) <= tol, k
    s.close()


# BF16 form: the uncut contraction runs on bf16 matrix cores with both operands split
# into bf16 hi + lo parts (four products, FP32 accumulation).  The split keeps 16 bits of
# each operand: a relative operand error of 2^-17 against 2^-24 for FP32, 128 times
# larger.  The FP32 runs of these cases stay below 4e-6, so the bar is 128 x 4e-6 = 5e-4
# (measured: 8.6e-5 on C1, 2.1e-4 on the elastic case).
BF16_TOL = 5e-4


def test_bf16_c1_parity(c1):
    cfg, disc, dt = c1
    s = _solver(cfg, "bf16")
    got = _run_gpu(s, cfg, dt, 500, [500])
    ref = timestep.cdm(disc, dt, 500, sources=cfg["sources"])["u"]
    assert rel_l2(got[500], ref) <= BF16_TOL
    s.close()


def test_bf16_elastic_3d_parity():
    # 5^3 cells, p=2, one ball: 102 uncut cells on the bf16 path, 23 cut cells
    cfg = workloads._base(3, (5, 5, 5), 2, [(0.55, 0.5, 0.5)], [0.2], ncomp=3, nsteps=100)
    cfg["sources"] = [dict(x=(0.1, 0.1, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)]
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    ref = timestep.cdm(disc, dt, 100, sources=cfg["sources"])["u"]
    for precision, tol in (("fp32", 1e-4), ("bf16", BF16_TOL)):
        s = _solver(cfg, precision)
        got = _run_gpu(s, cfg, dt, 100, [100])
        assert rel_l2(got[100], ref) <= tol, precision
        s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_every_tile_configuration(c2_small, precision, tol):
    # every kernel the autotuner may choose (2-D tile kernels, streaming kernels, generic
    # tile shapes) against the oracle on the same 64^2 p=4 problem
    from paper_2501_19013_amd import fcw
    cfg, disc, dt = c2_small
    ref = timestep.cdm(disc, dt, 60, sources=cfg["sources"])["u"]
    s = _solver(cfg, precision)
    confs = s.tile_configs()
    assert len(confs) >= 5
    for i, conf in enumerate(confs):
        s.select_tile(i)
        got = _run_gpu(s, cfg, dt, 60, [25, 35])
        assert rel_l2(got[60], ref) <= tol, (i, conf)
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4), ("bf16", BF16_TOL)])
def test_elastic_3d_every_tile_configuration(precision, tol):
    # every 3-D elastic tile shape and block size the autotuner may choose, on a 9x6x5 p=2
    # grid with one ball (several tiles per axis, ragged edge tiles, cut cells)
    cfg = workloads._base(3, (9, 6, 5), 2, [(0.45, 0.3, 0.25)], [0.15], ncomp=3, nsteps=60,
                          hi=(0.9, 0.6, 0.5))
    cfg["sources"] = [dict(x=(0.1, 0.1, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)]
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    ref = timestep.cdm(disc, dt, 60, sources=cfg["sources"])["u"]
    s = _solver(cfg, precision)
    confs = s.tile_configs()
    assert len(confs) >= 2
    for i, conf in enumerate(confs):
        s.select_tile(i)
        got = _run_gpu(s, cfg, dt, 60, [60])
        assert rel_l2(got[60], ref) <= tol, (i, conf)
    s.close()


def _elastic_p3():
    # 3-D elastic p = 3 (n_loc = 192) on a ragged 5x4x3 grid with one ball: two tiles per
    # axis of the 4x2x2 and 4x4x2 tile shapes, cut cells
    cfg = workloads._base(3, (5, 4, 3), 3, [(0.3, 0.22, 0.16)], [0.12], ncomp=3, nsteps=40,
                          hi=(0.5, 0.4, 0.3), tree_depth=2)
    cfg["sources"] = [dict(x=(0.05, 0.05, 0.05), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)]
    return cfg


def test_elastic_3d_p3_setup_parity():
    cfg = _elastic_p3()
    disc = _oracle(cfg)
    assert disc.prob.n_loc == 192 and len(disc.cut_cells) > 0
    s = _solver(cfg, "fp64")
    _setup_parity(cfg, disc, s)
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_elastic_3d_p3_every_tile_configuration(precision, tol):
    cfg = _elastic_p3()
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    ref = timestep.cdm(disc, dt, 40, sources=cfg["sources"])["u"]
    s = _solver(cfg, precision)
    confs = s.tile_configs()
    assert len(confs) >= 1
    for i, conf in enumerate(confs):
        s.select_tile(i)
        got = _run_gpu(s, cfg, dt, 40, [15, 25])
        assert rel_l2(got[40], ref) <= tol, (i, conf)
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_elastic_3d_p3_multi_rhs(precision, tol):
    # three right-hand sides in one call (the cut products of 192-row cells on the matrix
    # cores), each against its own oracle run, every tile configuration
    import torch
    cfg = _elastic_p3()
    srcs = [cfg["sources"][0],
            dict(x=(0.45, 0.05, 0.25), dir=(0.0, 0.6, 0.8), f0=14.0, amp=-0.7),
            dict(x=(0.1, 0.35, 0.2), dir=(0.0, 0.0, 1.0), f0=8.0, amp=0.4)]
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    refs = [timestep.cdm(disc, dt, 40, sources=[q])["u"] for q in srcs]
    s = _solver(cfg, precision)
    for i, conf in enumerate(s.tile_configs()):
        s.select_tile(i)
        u, d = s.zeros(len(srcs)), s.zeros(len(srcs))
        s.step(u, d, srcs, dt, 15, start=True)
        s.step(u, d, srcs, dt, 25, t0=15 * dt)
        torch.cuda.synchronize()
        got = u.double().cpu().numpy()
        for q in range(len(srcs)):
            assert rel_l2(got[q], refs[q]) <= tol, (i, conf, q)
    s.close()


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_scalar_3d_every_tile_configuration(p, precision, tol):
    # every 3-D scalar tile shape the autotuner may choose, on a ragged 9x7x5 grid with one
    # ball (several tiles per axis, edge tiles, cut cells)
    cfg = workloads._base(3, (9, 7, 5), p, [(0.5, 0.35, 0.25)], [0.17], nsteps=50,
                          hi=(0.9, 0.7, 0.5), tree_depth=2)
    disc = _oracle(cfg)
    assert len(disc.cut_cells) > 0
    dt = 0.9 * timestep.critical_dt(disc)
    ref = timestep.cdm(disc, dt, 50, sources=cfg["sources"])["u"]
    s = _solver(cfg, precision)
    confs = s.tile_configs()
    assert len(confs) >= 2
    for i, conf in enumerate(confs):
        s.select_tile(i)
        got = _run_gpu(s, cfg, dt, 50, [21, 29])
        assert rel_l2(got[50], ref) <= tol, (i, conf)
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_elastic_3d_multi_rhs(precision, tol):
    # three right-hand sides (sources in other places and directions) in one call, each
    # against its own oracle run
    import torch
    cfg = workloads.scaled_config(3, 5, 2, seed=4, ncomp=3, porosity=0.15)
    srcs = [dict(x=(0.1, 0.1, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0),
            dict(x=(0.72, 0.33, 0.61), dir=(0.0, 0.6, 0.8), f0=14.0, amp=-0.7),
            dict(x=(0.45, 0.85, 0.2), dir=(0.0, 0.0, 1.0), f0=8.0, amp=0.4)]
    srcs = [q for q in srcs if not np.any(np.linalg.norm(cfg["void_center"] - q["x"], axis=1)
                                          < cfg["void_radius"])]
    assert len(srcs) >= 2
    disc = _oracle(cfg)
    dt = 0.9 * timestep.critical_dt(disc)
    nsteps = 70
    s = _solver(cfg, precision)
    u, d = s.zeros(len(srcs)), s.zeros(len(srcs))
    s.step(u, d, srcs, dt, 33, start=True)
    s.step(u, d, srcs, dt, nsteps - 33, t0=33 * dt)
    torch.cuda.synchronize()
    got = u.double().cpu().numpy()
    for q, src in enumerate(srcs):
        ref = timestep.cdm(disc, dt, nsteps, sources=[src])["u"]
        assert rel_l2(got[q], ref) <= tol, (q, rel_l2(got[q], ref))
    s.close()


def test_error_paths():
    from paper_2501_19013_amd import fcw
    cfg = workloads.config("c1")
    s = _solver(cfg, "fp64")
    u, d = s.zeros(1), s.zeros(1)
    with pytest.raises(fcw.FcwError) as e:     # source inside the hole
        s.step(u, d, [dict(x=(0.5, 0.5), f0=10.0)], 1e-3, 3, start=True)
    assert e.value.status == fcw.FCW_E_ARG
    with pytest.raises(fcw.FcwError) as e:     # outside the box
        s.step(u, d, [dict(x=(1.5, 0.5), f0=10.0)], 1e-3, 3, start=True)
    assert e.value.status == fcw.FCW_E_ARG
    with pytest.raises(fcw.FcwError) as e:     # implicit DOFs but no v_c, a_c
        fcw.step_imex(s.ctx, 1, u, d, None, None, None, 0.0, 1e-3, 1, 1)
    assert e.value.status == fcw.FCW_E_ARG
    s.step(u, d, None, 1e-3, 0)               # zero steps is a no-op
    s.close()
    s = _solver(cfg, "fp32")                   # the IMEX scheme is FP64 only
    u, d = s.zeros(1), s.zeros(1)
    with pytest.raises(fcw.FcwError) as e:
        fcw.step_imex(s.ctx, 1, u, d, None, None, None, 0.0, 1e-3, 1, 1)
    assert e.value.status == fcw.FCW_E_UNSUPPORTED
    s.close()


def test_bitwise_reproducible(c1):
    import torch
    cfg, _, dt = c1
    outs = []
    for _ in range(2):
        s = _solver(cfg, "fp32")
        u, d = s.run(cfg["sources"], dt, 300)
        torch.cuda.synchronize()
        outs.append(u.cpu().numpy().copy())
        s.close()
    assert np.array_equal(outs[0], outs[1])
