"""Parity of the semi-explicit (IMEX) step (Sec. 2.5, Alg. imex) with the FP64 oracle.

The implicit DOF set must equal the oracle's exactly (an index set).  The states after
the steps agree to a tolerance set by the conditioning of S = M^cc + dt^2/4 K^cc:

* with alpha = 1e-4 in the voids, cond(S) is about 3e5 on the C1 geometry and the
  oracle's own result moves by 1e-14 when its cut-cell matrices move by 1e-14, so the
  device (dense Cholesky in another order, its own tree quadrature) must agree to 1e-10;
* with the paper's alpha = 1e-12, cut-cell fragments of almost no material make
  cond(S) about 6e12: a relative change of 1e-15 in the cut-cell matrices (rounding of
  the quadrature sums) moves the oracle's result by 6e-7, so the bar there is 1e-5.
"""
import numpy as np
import pytest

import workloads
from oracle import imex as ox
from oracle import problem, timestep

pytestmark = pytest.mark.gpu

TOL = 1e-10       # alpha = 1e-4
TOL_ILL = 1e-5    # alpha = 1e-12


def _run(cfg, dt, chunks, sources, autotune=False):
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    s = Solver(cfg, precision="fp64")
    if autotune:
        s.autotune(nrhs=len(sources), nsteps=10)
    nc = fcw.imex_prepare(s.ctx, dt)
    dofs = fcw.export(s.ctx, fcw.ARR_IMEX_DOFS)
    nrhs = len(sources)
    u, d = s.zeros(nrhs), s.zeros(nrhs)
    v = torch.zeros(nrhs, max(nc, 1), dtype=torch.float64, device="cuda")
    a = torch.zeros_like(v)
    k = 0
    for n in chunks:
        fcw.step_imex(s.ctx, nrhs, u, d, v, a, sources, k * dt, dt, n, int(k == 0))
        k += n
    torch.cuda.synchronize()
    out = dict(u=u.double().cpu().numpy(), v=v.cpu().numpy()[:, :nc], a=a.cpu().numpy()[:, :nc],
               dofs=dofs, nc=nc, layout=fcw.imex_layout(s.ctx))
    s.close()
    return out


def _check(cfg, steps, chunks, sources, dt=None, tol=TOL, disc=None, sparse=False,
           autotune=False):
    if disc is None:
        disc = problem.build(problem.Problem.from_config(cfg))
    if dt is None:
        dt = 0.9 * timestep.critical_dt(disc)
    got = _run(cfg, dt, chunks, sources, autotune=autotune)
    c, _ = ox.partition(disc)
    assert got["nc"] == len(c)
    assert np.array_equal(got["dofs"], c)
    for r, src in enumerate(sources):
        ref = ox.imex(disc, dt, steps, sources=[src], sparse=sparse)
        assert np.linalg.norm(ref["u"]) > 0
        e = np.linalg.norm(got["u"][r] - ref["u"]) / np.linalg.norm(ref["u"])
        ev = np.linalg.norm(got["v"][r] - ref["v_c"]) / max(np.linalg.norm(ref["v_c"]), 1e-300)
        assert e <= tol and ev <= tol, (r, e, ev)
    return got


def _c1(alpha):
    cfg = workloads.config("c1")
    cfg["alpha"] = alpha
    return cfg


def test_imex_c1_parity():
    # 2-D p=3, 16x16 cells, one circular hole; two calls (start, then continue)
    cfg = _c1(1e-4)
    _check(cfg, 200, [120, 80], cfg["sources"])


def test_imex_c1_paper_alpha():
    cfg = _c1(1e-12)
    _check(cfg, 200, [200], cfg["sources"], tol=TOL_ILL)


def test_imex_two_sources_batched():
    cfg = _c1(1e-4)
    srcs = [dict(x=(0.1, 0.1), f0=10.0, amp=1.0), dict(x=(0.83, 0.27), f0=7.0, amp=0.5)]
    _check(cfg, 90, [90], srcs)


def test_imex_ten_sources():
    # ten right-hand sides (each tile of S^-1 is read once for all of them)
    cfg = _c1(1e-4)
    xs = [(0.1, 0.1), (0.9, 0.1), (0.1, 0.9), (0.9, 0.9), (0.5, 0.08), (0.08, 0.5),
          (0.92, 0.5), (0.5, 0.92), (0.25, 0.75), (0.75, 0.25)]
    srcs = [dict(x=x, f0=8.0 + i, amp=1.0) for i, x in enumerate(xs)]
    _check(cfg, 50, [30, 20], srcs)


def test_imex_3d_scalar_parity():
    cfg = workloads._base(3, (5, 4, 4), 2, [(0.52, 0.4, 0.4)], [0.22], nsteps=60,
                          hi=(1.0, 0.8, 0.8), alpha=1e-4)
    cfg["sources"] = [dict(x=(0.1, 0.1, 0.1), f0=8.0, amp=1.0)]
    _check(cfg, 60, [60], cfg["sources"])


def test_imex_3d_elastic_parity():
    cfg = workloads._base(3, (4, 4, 4), 2, [(0.55, 0.5, 0.5)], [0.2], ncomp=3, nsteps=40,
                          alpha=1e-4)
    cfg["sources"] = [dict(x=(0.1, 0.1, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)]
    _check(cfg, 40, [40], cfg["sources"])


def test_imex_3d_elastic_p3_parity():
    # 3-D elastic p = 3 (192 DOFs per cell, 1 029 stencil slots per implicit row of K)
    cfg = workloads._base(3, (5, 4, 3), 3, [(0.3, 0.22, 0.16)], [0.12], ncomp=3, nsteps=30,
                          hi=(0.5, 0.4, 0.3), tree_depth=2, alpha=1e-4)
    cfg["sources"] = [dict(x=(0.05, 0.05, 0.05), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0),
                      dict(x=(0.45, 0.05, 0.25), dir=(0.0, 0.6, 0.8), f0=14.0, amp=-0.7)]
    _check(cfg, 30, [12, 18], cfg["sources"])


def test_imex_3d_elastic_two_blocks():
    """Two pores far enough apart that no active cell holds implicit nodes of both: two
    blocks of coupled DOFs, each with the three components of its nodes (the block order
    permutes the component-major implicit DOFs)."""
    cfg = workloads._base(3, (8, 4, 4), 2, [(0.4, 0.5, 0.5), (1.6, 0.5, 0.5)], [0.2, 0.2],
                          ncomp=3, nsteps=40, hi=(2.0, 1.0, 1.0), alpha=1e-4)
    cfg["sources"] = [dict(x=(1.0, 0.3, 0.3), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0),
                      dict(x=(1.1, 0.6, 0.7), dir=(0.0, 0.0, 1.0), f0=12.0, amp=0.5)]
    got = _check(cfg, 40, [15, 25], cfg["sources"])
    assert got["layout"]["n_blocks"] == 2


def test_imex_implicit_set_above_the_dense_block_limit():
    """A 2-D p = 4 field of 50 voids on 96 x 96 cells: 19 815 implicit DOFs, more than one
    dense block may hold (FCW_IMEX_MAX_NC).  The device splits them into blocks of coupled
    DOFs (the cut cells around one void or cluster of voids, linked through shared cells);
    the oracle solves with a sparse LU factor of the whole S.  Two right-hand sides, two
    calls."""
    import re
    from pathlib import Path
    cc, rr = workloads.random_circles(seed=5, count=50, rmin=0.02, rmax=0.04)
    cfg = workloads._base(2, (96, 96), 4, cc, rr, alpha=1e-4)
    disc = problem.build(problem.Problem.from_config(cfg))
    c, d = ox.partition(disc)
    header = (Path(__file__).resolve().parents[1] / "include" / "fcw.h").read_text()
    limit = int(re.search(r"#define FCW_IMEX_MAX_NC (\d+)", header).group(1))
    assert len(c) > limit
    # a step below the explicit block's limit (Gershgorin bound of (M^dd)^-1 K^dd)
    K = problem.assembled_K(disc).tocsr()
    im = disc.inv_mass_dof()
    g = np.asarray(abs(K[d][:, d]).sum(axis=1)).ravel() * im[d]
    dt = 0.8 * 2.0 / np.sqrt(g.max())
    srcs = [dict(x=(0.1, 0.1), f0=45.0, amp=1.0), dict(x=(0.85, 0.6), f0=60.0, amp=0.7)]
    got = _check(cfg, 80, [30, 50], srcs, dt=dt, disc=disc, sparse=True)
    lay = got["layout"]
    assert 1 < lay["n_blocks"] and lay["largest"] <= limit
    # each block's packed upper tiles: far less than one dense inverse of the whole set
    assert lay["solve_bytes"] < 0.25 * 8 * len(c) ** 2


def test_imex_with_the_autotuned_explicit_kernel():
    """The explicit part runs whichever step kernel the context has selected (here the one
    the autotuner picks on the void field at 64 x 64 cells, p = 3); one and two right-hand
    sides."""
    cc, rr = workloads.random_circles(seed=2)
    cfg = workloads._base(2, (64, 64), 3, cc, rr, alpha=1e-4)
    disc = problem.build(problem.Problem.from_config(cfg))
    c, d = ox.partition(disc)
    K = problem.assembled_K(disc).tocsr()
    im = disc.inv_mass_dof()
    g = np.asarray(abs(K[d][:, d]).sum(axis=1)).ravel() * im[d]
    dt = 0.8 * 2.0 / np.sqrt(g.max())
    srcs = [dict(x=(0.1, 0.1), f0=20.0, amp=1.0), dict(x=(0.7, 0.45), f0=25.0, amp=0.5)]
    for batch in (srcs[:1], srcs):
        _check(cfg, 60, [20, 40], batch, dt=dt, disc=disc, sparse=True, autotune=True)


def test_imex_without_cut_cells_is_the_explicit_step():
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg = workloads._base(2, (12, 12), 3, np.zeros((0, 2)), np.zeros(0), nsteps=50)
    src = [dict(x=(0.3, 0.4), f0=10.0, amp=1.0)]
    s = Solver(cfg, precision="fp64")
    dt = 0.9 * s.critical_dt(max_iter=600, rtol=1e-9)
    assert fcw.imex_prepare(s.ctx, dt) == 0
    u1, d1 = s.zeros(1), s.zeros(1)
    fcw.step_imex(s.ctx, 1, u1, d1, None, None, src, 0.0, dt, 50, 1)
    u2, d2 = s.zeros(1), s.zeros(1)
    s.step(u2, d2, src, dt, 50, t0=0.0, start=True)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    s.close()


def test_imex_beyond_the_explicit_limit():
    # eps = 0: the lumped explicit step is limited by a tiny cut fragment; IMEX runs at
    # the step size of the uncut cells and matches the oracle there
    cfg = workloads._base(2, (6, 6), 2, [(0.5, 0.5)], [0.4949], eps=0.0, nsteps=300)
    cfg_u = workloads._base(2, (6, 6), 2, np.zeros((0, 2)), np.zeros(0))
    disc_u = problem.build(problem.Problem.from_config(cfg_u))
    dt = 0.9 * timestep.critical_dt(disc_u)
    src = [dict(x=(0.05, 0.05), f0=10.0, amp=1.0)]
    got = _check(cfg, 300, [300], src, dt=dt, tol=TOL_ILL)
    assert np.all(np.isfinite(got["u"]))


def _consistent_dt(disc):
    """0.9 * 2 / sqrt(lambda_max(M^-1 K)) for the block mass diag(M^dd, M^cc) (dense)."""
    c, d = ox.partition(disc)
    m_dd, Mcc = ox.mass_matrices(disc, c, d)
    act = np.concatenate([d, c])
    n = len(act)
    M = np.zeros((n, n))
    M[:len(d), :len(d)] = np.diag(m_dd)
    M[len(d):, len(d):] = Mcc.toarray()
    K = problem.assembled_K(disc)[act][:, act].toarray()
    Li = np.linalg.inv(np.linalg.cholesky(M))
    lam = np.linalg.eigvalsh(Li @ K @ Li.T)[-1]
    return 0.9 * 2.0 / np.sqrt(lam)


@pytest.mark.parametrize("alpha,tol", [(1e-4, 1e-10), (1e-12, 1e-8)])
def test_consistent_mass_cdm_parity(alpha, tol):
    # central differences with the consistent cut-DOF mass, C1, two calls; the bar at
    # alpha = 1e-12 follows from the oracle's own sensitivity (a 1e-15 relative change of
    # the cut-cell matrices moves its result by 1e-11)
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg = _c1(alpha)
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = _consistent_dt(disc)
    ref = ox.cdm_consistent(disc, dt, 200, sources=cfg["sources"])["u"]
    s = Solver(cfg, precision="fp64")
    u, d = s.zeros(1), s.zeros(1)
    fcw.step_consistent(s.ctx, 1, u, d, cfg["sources"], 0.0, dt, 120, 1)
    fcw.step_consistent(s.ctx, 1, u, d, cfg["sources"], 120 * dt, dt, 80, 0)
    torch.cuda.synchronize()
    got = u[0].cpu().numpy()
    s.close()
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)


def test_consistent_mass_cdm_3d_elastic():
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg = workloads._base(3, (4, 4, 4), 2, [(0.55, 0.5, 0.5)], [0.2], ncomp=3, nsteps=40,
                          alpha=1e-4)
    cfg["sources"] = [dict(x=(0.1, 0.1, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)]
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = _consistent_dt(disc)
    ref = ox.cdm_consistent(disc, dt, 40, sources=cfg["sources"])["u"]
    s = Solver(cfg, precision="fp64")
    u, d = s.zeros(1), s.zeros(1)
    fcw.step_consistent(s.ctx, 1, u, d, cfg["sources"], 0.0, dt, 40, 1)
    torch.cuda.synchronize()
    got = u[0].cpu().numpy()
    s.close()
    assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)
