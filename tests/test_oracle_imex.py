"""Pins of the IMEX oracle (Sec. 2.5, Alg. imex) and of central differences with the
consistent cut-DOF mass, against what the mathematics fixes:

* no cut cell: the scheme is central differences (eq. cdm with the Newmark start-up);
* every active DOF implicit and no load: the trapezoidal rule conserves the energy
  1/2 v^T M v + 1/2 u^T K u exactly;
* mixed split: second-order convergence in dt;
* stability set by the explicit part: without eigenvalue stabilisation the lumped
  explicit step diverges at the step size of the uncut cells, IMEX does not;
* consistent-mass central differences: eq. cdm without cut cells; the discrete energy
  with the block mass is conserved below 2 / sqrt(lambda_max(M^-1 K)) and grows above it.
"""
import numpy as np
import pytest

import workloads
from oracle import imex as ox
from oracle import problem, timestep


def _disc(centers, radii, n=6, p=2, eps=1e-4, alpha=1e-12):
    cfg = workloads._base(2, (n, n), p, centers, radii, eps=eps, alpha=alpha)
    return cfg, problem.build(problem.Problem.from_config(cfg))


def test_no_cut_cell_is_central_differences():
    cfg, disc = _disc(np.zeros((0, 2)), np.zeros(0))
    assert len(disc.cut_cells) == 0
    dt = 0.9 * timestep.critical_dt(disc)
    src = [dict(x=(0.31, 0.42), f0=10.0, amp=1.0)]
    got = ox.imex(disc, dt, 40, sources=src)
    ref = timestep.cdm(disc, dt, 40, sources=src)["u"]
    assert len(got["c"]) == 0
    assert np.linalg.norm(got["u"] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_all_implicit_conserves_energy():
    cfg, disc = _disc([(0.5, 0.5)], [0.21])
    c, d = ox.partition(disc)
    allc = np.sort(np.concatenate([c, d]))
    split = (allc, np.zeros(0, dtype=np.int64))
    m_dd, M = ox.mass_matrices(disc, *split)
    K = problem.assembled_K(disc)[allc][:, allc]
    rng = np.random.default_rng(7)
    u0 = np.zeros(disc.prob.ndof)
    u0[allc] = rng.standard_normal(len(allc))
    dt = 0.05  # far above any explicit limit: the trapezoidal rule is unconditionally stable
    e0 = 0.5 * u0[allc] @ (K @ u0[allc])
    for n in (10, 37):
        r = ox.imex(disc, dt, n, split=split, u0=u0)
        uc = r["u"][allc]
        e = 0.5 * r["v_c"] @ (M @ r["v_c"]) + 0.5 * uc @ (K @ uc)
        assert abs(e - e0) <= 1e-11 * e0, (n, e, e0)


def test_mixed_split_second_order():
    cfg, disc = _disc([(0.47, 0.52)], [0.23])
    c, d = ox.partition(disc)
    assert len(c) > 0 and len(d) > 0
    src = [dict(x=(0.1, 0.1), f0=6.0, amp=1.0)]
    dt0 = 0.5 * timestep.critical_dt(disc)
    T = 64 * dt0
    sol = {}
    for m in (1, 2, 4, 16):
        dt = dt0 / m
        sol[m] = ox.imex(disc, dt, int(round(T / dt)), sources=src)["u"]
    e1 = np.linalg.norm(sol[1] - sol[16])
    e2 = np.linalg.norm(sol[2] - sol[16])
    e4 = np.linalg.norm(sol[4] - sol[16])
    assert e1 > 0 and 3.0 < e1 / e2 < 5.5 and 3.0 < e2 / e4 < 5.5, (e1, e2, e4)


def test_stability_set_by_explicit_part():
    # eps = 0: no eigenvalue stabilisation, so a tiny cut fragment makes the lumped
    # explicit step unstable at the step size that the uncut cells allow
    centers, radii = [(0.5, 0.5)], [0.4949]
    cfg, disc = _disc(centers, radii, n=6, p=2, eps=0.0)
    cfg_u, disc_u = _disc(np.zeros((0, 2)), np.zeros(0), n=6, p=2)
    dt = 0.9 * timestep.critical_dt(disc_u)
    assert dt > timestep.critical_dt(disc)
    src = [dict(x=(0.05, 0.05), f0=10.0, amp=1.0)]
    n = 400
    r = ox.imex(disc, dt, n, sources=src)
    e = timestep.cdm(disc, dt, n, sources=src)["u"]
    assert np.all(np.isfinite(r["u"])) and np.abs(r["u"]).max() < 1e3
    assert not np.all(np.isfinite(e)) or np.abs(e).max() > 1e6


def test_consistent_cdm_without_cut_cells_is_cdm():
    cfg, disc = _disc(np.zeros((0, 2)), np.zeros(0))
    dt = 0.9 * timestep.critical_dt(disc)
    src = [dict(x=(0.31, 0.42), f0=10.0, amp=1.0)]
    got = ox.cdm_consistent(disc, dt, 40, sources=src)["u"]
    ref = timestep.cdm(disc, dt, 40, sources=src)["u"]
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def _block_mass(disc):
    c, d = ox.partition(disc)
    m_dd, Mcc = ox.mass_matrices(disc, c, d)
    act = np.concatenate([d, c])
    M = np.zeros((len(act), len(act)))
    M[:len(d), :len(d)] = np.diag(m_dd)
    M[len(d):, len(d):] = Mcc.toarray()
    K = problem.assembled_K(disc)[act][:, act].toarray()
    return act, M, K


def test_consistent_cdm_energy_and_stability_limit():
    # with the consistent cut-DOF mass the discrete CDM energy
    # 1/2 v^T M v + 1/2 u_{k+1}^T K u_k (v = (u_{k+1} - u_k) / dt) is conserved without load
    # below 2 / sqrt(lambda_max(M^-1 K)), and the step grows above it
    cfg, disc = _disc([(0.5, 0.5)], [0.4949], eps=0.0)
    act, M, K = _block_mass(disc)
    lam = float(np.max(np.real(np.linalg.eigvals(np.linalg.solve(M, K)))))
    dtc = 2.0 / np.sqrt(lam)
    rng = np.random.default_rng(3)
    u0 = np.zeros(disc.prob.ndof)
    u0[act] = rng.standard_normal(len(act))
    es = []
    for n in (30, 31, 90, 91):
        r = ox.cdm_consistent(disc, 0.9 * dtc, n, u0=u0)
        v = (r["u"][act] - r["u_prev"][act]) / (0.9 * dtc)
        es.append(0.5 * v @ M @ v + 0.5 * r["u"][act] @ K @ r["u_prev"][act])
    assert max(es) - min(es) <= 1e-10 * abs(es[0]), es
    grow = ox.cdm_consistent(disc, 1.05 * dtc, 600, u0=u0)["u"]
    assert np.abs(grow).max() > 1e3 * np.abs(u0).max()


def _newmark_predictor_corrector(disc, split, dt, nsteps, src, beta=0.25, gamma=0.5):
    """The implicit DOFs in the predictor-corrector (acceleration) form of the Newmark
    relations, the explicit DOFs by central differences: an independent arrangement of
    the same scheme as the oracle's displacement form."""
    import scipy.linalg as sla
    prob = disc.prob
    c, d = split
    m_dd, Mcc = ox.mass_matrices(disc, c, d)
    K = problem.assembled_K(disc).toarray()
    loads = [(problem.load_vector(disc, s), s["f0"]) for s in src]

    def F(k):
        out = np.zeros(prob.ndof)
        for b, f0 in loads:
            out += problem.ricker(k * dt, f0) * b
        return out

    M = Mcc.toarray()
    u = np.zeros(prob.ndof)
    v = np.zeros(len(c))
    a = np.linalg.solve(M, F(0)[c] - K[c] @ u) if len(c) else np.zeros(0)
    prev_d = None
    for k in range(nsteps):
        nd = u[d] + (0.5 if k == 0 else 1.0) * dt * dt * (F(k)[d] - K[d] @ u) / m_dd
        if k > 0:
            nd = nd + (u[d] - prev_d)
        prev_d = u[d].copy()
        pred = u.copy()
        pred[d] = nd
        if len(c):
            pred[c] = u[c] + dt * v + (0.5 - beta) * dt * dt * a
            vp = v + (1.0 - gamma) * dt * a
            a = np.linalg.solve(M + beta * dt * dt * K[np.ix_(c, c)], F(k + 1)[c] - K[c] @ pred)
            v = vp + gamma * dt * a
            pred[c] += beta * dt * dt * a
        u = pred
    return u, v, a


@pytest.mark.parametrize("mode", ["mixed", "all_implicit"])
def test_displacement_form_equals_predictor_corrector(mode):
    cfg, disc = _disc([(0.47, 0.52)], [0.23], alpha=1e-4)
    c, d = ox.partition(disc)
    if mode == "all_implicit":
        c = np.sort(np.concatenate([c, d]))
        d = np.zeros(0, dtype=np.int64)
    src = [dict(x=(0.1, 0.1), f0=10.0, amp=1.0)]
    dt = 0.5 * timestep.critical_dt(disc) if mode == "mixed" else 0.01
    got = ox.imex(disc, dt, 60, sources=src, split=(c, d))
    u, v, a = _newmark_predictor_corrector(disc, (c, d), dt, 60, src)
    assert np.linalg.norm(got["u"] - u) <= 1e-9 * np.linalg.norm(u)
    assert np.linalg.norm(got["v_c"] - v) <= 1e-8 * np.linalg.norm(v)


def test_implicit_set_of_the_3d_imex_workload_exceeds_the_dense_limit():
    """Size and blocks of the implicit set (every component of the nodes of cut cells,
    Sec. 2.5) of the 3-D elastic IMEX workload (64^3 cells, p = 3, the spherical-pore
    field), from the oracle's cell classes.  S couples two implicit nodes when an active
    cell holds both; at porosity 0.2 nearly all implicit nodes fall into one such block,
    far above the dense block limit of the device's IMEX set-up, so this workload needs a
    sparse factorisation of S."""
    import itertools
    import re
    from pathlib import Path

    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    import workloads
    from oracle import geometry
    from oracle.problem import Problem
    cfg = workloads.config("c4")
    prob = Problem.from_config(cfg)
    cls = geometry.classify_cells(prob)
    n, p = prob.ncells, prob.p
    npts = [k * p + 1 for k in n]

    def cell_nodes(cells):
        ix = [cells % n[0], (cells // n[0]) % n[1], cells // (n[0] * n[1])]
        return np.stack([(ix[0] * p + a) + npts[0] * ((ix[1] * p + b) + npts[1] * (ix[2] * p + c))
                         for c, b, a in itertools.product(range(p + 1), repeat=3)], 1)

    cut_nodes = cell_nodes(np.flatnonzero(cls == geometry.CUT))
    imp = np.unique(cut_nodes)
    n_c = 3 * imp.size
    header = (Path(__file__).resolve().parents[1] / "include" / "fcw.h").read_text()
    limit = int(re.search(r"#define FCW_IMEX_MAX_NC (\d+)", header).group(1))
    # blocks: implicit nodes linked through every active (cut or uncut) cell
    rows, cols = [], []
    for cells in (np.flatnonzero(cls == geometry.CUT), np.flatnonzero(cls == geometry.UNCUT)):
        nodes = cell_nodes(cells)
        pos = np.minimum(np.searchsorted(imp, nodes), imp.size - 1)
        hit = imp[pos] == nodes
        first = np.where(hit.any(1), pos[np.arange(len(pos)), hit.argmax(1)], -1)
        keep = hit & (first[:, None] >= 0)
        rows.append(np.broadcast_to(first[:, None], pos.shape)[keep])
        cols.append(pos[keep])
    r, c = np.concatenate(rows), np.concatenate(cols)
    g = coo_matrix((np.ones(r.size), (r, c)), shape=(imp.size, imp.size))
    nblk, lab = connected_components(g, directed=False)
    largest = 3 * int(np.bincount(lab).max())
    assert n_c > 100 * limit and largest > 100 * limit, (n_c, largest)
    assert largest > 0.9 * n_c
    print(f"cut cells {int((cls == geometry.CUT).sum())}, implicit DOFs {n_c}, "
          f"blocks {nblk}, largest {largest}")


def test_sparse_and_dense_solves_agree():
    """The sparse-LU variant of the oracle's IMEX solves (for large implicit sets) gives the
    dense-Cholesky result: the same equations, another factorisation (alpha = 1e-4, where
    S is well conditioned)."""
    cfg = workloads.config("c1")
    cfg["alpha"] = 1e-4
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = 0.9 * timestep.critical_dt(disc)
    a = ox.imex(disc, dt, 30, sources=cfg["sources"])
    b = ox.imex(disc, dt, 30, sources=cfg["sources"], sparse=True)
    assert len(a["c"]) > 0
    for key in ("u", "v_c", "a_c"):
        assert np.linalg.norm(a[key] - b[key]) <= 1e-9 * np.linalg.norm(a[key]), key
