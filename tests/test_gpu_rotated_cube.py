"""GPU parity on the paper's benchmark geometry (Sec. 3.1): the rotated cube of edge 0.3
in the cube of edge 0.5, through the C ABI.

* cell classes bit for bit against the oracle, and the active-DOF counts of Table
  timing_discretizations (the eleven the exact overlap test reproduces, and the four
  others at the offsets the oracle's pins name);
* cut-cell stiffness and mass against the oracle's tree quadrature;
* observer traces at the 11 points of Table observer_locations (on the cube's faces,
  edges and corners) for a point source inside the cube, FP64 within 1e-10 and FP32
  within 1e-4 of the largest trace value, against the oracle's observer rows.
"""
import numpy as np
import pytest

import workloads
from oracle import geometry, problem, timestep

pytestmark = pytest.mark.gpu

TABLE = {(2, 28): 52353, (3, 13): 22816, (4, 9): 21109, (5, 7): 22706, (3, 18): 52375,
         (4, 12): 43065, (5, 9): 40176, (3, 20): 69391, (4, 15): 75085, (3, 19): 60472,
         (2, 31): 69083, (3, 14): 27793, (4, 10): 27233, (5, 11): 67086, (3, 31): 226108}
NOT_REPRODUCED = {(2, 28): 36, (3, 13): 72, (2, 31): 24, (3, 31): 72}


def _active_nodes(cls, prob):
    table = prob.cell_node_table()
    mark = np.zeros(prob.nnodes, dtype=bool)
    mark[table[cls != geometry.OUT].ravel()] = True
    return int(mark.sum())


@pytest.mark.parametrize("p,n", [(2, 28), (3, 13), (4, 9), (3, 18), (4, 12), (2, 31)])
def test_classes_and_dof_counts(p, n):
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    if p > 4:
        pytest.skip("3-D scalar step kernels are built for p <= 4")
    cfg = workloads.rotated_cube(n, p)
    prob = problem.Problem.from_config(cfg)
    ref = geometry.classify_cells(prob)
    s = Solver(cfg, precision="fp64")
    cls = s.export(fcw.ARR_CELL_CLASS)
    # a cut cell whose tree holds no physical box is dropped on the device (and by the
    # oracle's assembly); compare the classes before that with the oracle's predicate
    cand = s.export(fcw.ARR_CUT_CELLS)
    pre = cls.copy()
    pre[cand] = geometry.CUT
    np.testing.assert_array_equal(pre, ref)
    got = _active_nodes(cls, prob)
    assert got - TABLE[(p, n)] == NOT_REPRODUCED.get((p, n), 0), (p, n, got)
    s.close()


@pytest.fixture(scope="module")
def cube_p3():
    cfg = workloads.rotated_cube(10, 3, tree_depth=2)
    # a point source inside the cube near the face centre of the paper's source
    cfg["sources"] = [dict(x=tuple(workloads.cube_point(cfg, (-0.12, 0.01, -0.005))), f0=10.0,
                           amp=1.0)]
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = 0.9 * timestep.critical_dt(disc)
    return cfg, disc, dt


def test_cut_cell_matrices(cube_p3):
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, disc, _ = cube_p3
    s = Solver(cfg, precision="fp64")
    cls = s.export(fcw.ARR_CELL_CLASS)
    np.testing.assert_array_equal(cls, disc.cls)
    cand = s.export(fcw.ARR_CUT_CELLS)
    keep = cls[cand] == geometry.CUT
    np.testing.assert_array_equal(cand[keep], disc.cut_cells)
    nl, ns = disc.prob.n_loc, disc.prob.n_s
    kc = s.export(fcw.ARR_K_CUT).reshape(-1, nl, nl)[keep]
    mc = s.export(fcw.ARR_M_CUT).reshape(-1, ns, ns)[keep]
    for q in range(len(disc.cut_cells)):
        assert np.abs(kc[q] - disc.K_cut[q]).max() <= 1e-12 * np.abs(disc.K_cut[q]).max(), q
        assert np.abs(mc[q] - disc.Mo_cut[q]).max() <= 1e-13 * np.abs(disc.Mo_cut[q]).max(), q
    mass = s.export(fcw.ARR_MASS)
    np.testing.assert_allclose(mass, disc.mass, rtol=1e-10, atol=1e-10 * disc.mass.max())
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_observer_traces(cube_p3, precision, tol):
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, disc, dt = cube_p3
    obs = workloads.cube_observers(cfg)
    nsteps = 150
    s = Solver(cfg, precision=precision)
    u, d = s.zeros(1), s.zeros(1)
    tr = torch.full((1, nsteps + 1, len(obs), 1), float("nan"), dtype=torch.float64,
                    device="cuda")
    fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=cfg["sources"], dt=dt, nsteps=nsteps,
                  start=1, receivers=[tuple(x) for x in obs], traces=tr)])
    torch.cuda.synchronize()
    R = problem.receiver_rows(disc, obs)
    ref = timestep.cdm(disc, dt, nsteps, sources=cfg["sources"], receivers=R)["trace"]
    got = tr.cpu().numpy()[0, :, :, 0]
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(got - ref).max() <= tol * scale
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_gaussian_source_at_the_face_centre(precision, tol):
    """The benchmark's excitation (Sec. 3.1): a Gaussian of sigma = 0.01 centred on a face
    of the cube (half of it in the fictitious domain) with the Ricker pulse; the 11
    observer traces against the oracle's."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg = workloads.rotated_cube(10, 3, tree_depth=2)
    src = [dict(x=cfg["sources"][0]["x"], sigma=0.01, f0=10.0, amp=1.0)]
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = 0.9 * timestep.critical_dt(disc)
    obs = workloads.cube_observers(cfg)
    nsteps = 160
    s = Solver(cfg, precision=precision)
    u, d = s.zeros(1), s.zeros(1)
    tr = torch.full((1, nsteps + 1, len(obs), 1), float("nan"), dtype=torch.float64,
                    device="cuda")
    fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=src, dt=dt, nsteps=nsteps, start=1,
                  receivers=[tuple(x) for x in obs], traces=tr)])
    torch.cuda.synchronize()
    R = problem.receiver_rows(disc, obs)
    ref = timestep.cdm(disc, dt, nsteps, sources=src, receivers=R)
    got = tr.cpu().numpy()[0, :, :, 0]
    scale = np.abs(ref["trace"]).max()
    assert scale > 0
    assert np.abs(got - ref["trace"]).max() <= tol * scale
    uo = ref["u"]
    assert np.linalg.norm(u[0].double().cpu().numpy() - uo) <= tol * np.linalg.norm(uo)
    s.close()
