"""Pins of the oracle's time stepping and critical time step: closed-form eigen-mode
recurrence, continuum standing wave, exact discrete energy balance, reciprocity,
linearity, stability threshold and a closed-form lambda_max."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import workloads
from oracle import problem, timestep
from oracle.problem import Problem, apply_K, assembled_K, build, load_vector


def _box(dim, n, p, ncomp=1, **kw):
    cfg = workloads._base(dim, (n,) * dim, p, np.zeros((0, dim)), np.zeros(0), ncomp=ncomp, **kw)
    return build(Problem.from_config(cfg))


@pytest.fixture(scope="module")
def c1():
    cfg = workloads.config("c1")
    return cfg, build(Problem.from_config(cfg))


@pytest.mark.parametrize("n,c", [(4, 1.0), (8, 1.0), (8, 2.5)])
def test_lambda_max_bilinear_closed_form(n, c):
    # p = 1, uncut box, lumped mass, exact stiffness: the mode alternating in x and
    # constant in y is an exact eigenvector with lambda = 4 c^2 / h^2, the maximum,
    # hence dt_crit = h / c
    disc = _box(2, n, 1, c=c)
    h = disc.prob.h
    assert abs(timestep.lambda_max(disc) - 4 * c * c / h ** 2) < 1e-10 * 4 * c * c / h ** 2
    assert abs(timestep.critical_dt(disc) - h / c) < 1e-12


def test_lambda_max_dense_vs_lanczos(c1):
    _, disc = c1
    dense = timestep.lambda_max(disc)
    lanczos = timestep.lambda_max(disc, dense_limit=0)
    assert abs(dense - lanczos) < 1e-9 * dense


@pytest.mark.parametrize("p,n", [(2, 4), (3, 3), (4, 2)])
def test_spectral_convergence_of_lowest_mode(p, n):
    # lowest nonzero eigenvalue of the Neumann unit square -> (pi c)^2, error ~ h^(2p)
    errs = []
    for m in (n, 2 * n):
        disc = _box(2, m, p)
        K = assembled_K(disc).toarray()
        ev = sl.eigh(K, np.diag(disc.mass), eigvals_only=True, subset_by_index=[0, 2])
        errs.append(abs(ev[1] - math.pi ** 2) / math.pi ** 2)
    assert errs[0] < 1e-3
    assert errs[1] < errs[0] / 2 ** (2 * p - 1)


def test_eigenmode_recurrence_closed_form(c1):
    # u0 = phi (generalized eigenvector of (K, M)), v0 = 0, F = 0:
    # eq. cdm with the beta = 0 start-up gives u_k = phi cos(k theta) exactly,
    # cos(theta) = 1 - dt^2 lambda / 2
    _, disc = c1
    K = assembled_K(disc).toarray()
    act = disc.mass > 0
    Ka = K[np.ix_(act, act)]
    lam, vec = sl.eigh(Ka, np.diag(disc.mass[act]))
    dt = 0.9 * 2 / math.sqrt(lam[-1])
    for j in (1, 7, len(lam) // 2, len(lam) - 1):
        phi = np.zeros(disc.prob.ndof)
        phi[act] = vec[:, j] / np.abs(vec[:, j]).max()
        theta = math.acos(1 - dt * dt * lam[j] / 2)
        out = timestep.cdm(disc, dt, 60, u0=phi, checkpoints=(13, 60))
        for k in (13, 60):
            np.testing.assert_allclose(out["snapshots"][k], phi * math.cos(k * theta), atol=1e-10)


def test_standing_wave_continuum():
    # uncut unit square, u0 = cos(pi x) cos(2 pi y), v0 = 0: the continuum mode with
    # omega^2 = 5 pi^2 c^2, advanced by central differences, is u0 cos(k theta) with
    # cos(theta) = 1 - dt^2 omega^2 / 2; the spatial error of p = 4 is far smaller
    disc = _box(2, 8, 4, c=1.0)
    prob = disc.prob
    # 1-D node coordinates: GLL points mapped into each cell
    from oracle.basis import gll_points
    xi, _ = gll_points(prob.p)
    x = np.concatenate([[0.0]] + [k * prob.h + (xi[1:] + 1) * prob.h / 2
                                  for k in range(prob.ncells[0])])
    X, Y = np.meshgrid(x, x)  # rows = y
    u0 = (np.cos(math.pi * X) * np.cos(2 * math.pi * Y)).ravel()
    dt = 0.5 * timestep.critical_dt(disc)
    ns = int(round(0.3 / dt))
    out = timestep.cdm(disc, dt, ns, u0=u0)
    theta = math.acos(1 - dt * dt * 5 * math.pi ** 2 / 2)
    exact = u0 * math.cos(ns * theta)
    assert np.abs(out["u"] - exact).max() < 2e-6
    # and the time-continuous solution within the O(dt^2) phase error of the scheme
    assert np.abs(out["u"] - u0 * math.cos(math.pi * math.sqrt(5) * ns * dt)).max() < 1e-3


def test_energy_conserved_without_load(c1):
    _, disc = c1
    rng = np.random.default_rng(3)
    act = np.tile(disc.mass > 0, disc.prob.ncomp)
    u0 = rng.standard_normal(disc.prob.ndof) * act
    v0 = rng.standard_normal(disc.prob.ndof) * act
    dt = 0.9 * timestep.critical_dt(disc)
    E = []
    for k in (1, 2, 50, 51, 200):
        out = timestep.cdm(disc, dt, k, u0=u0, v0=v0)
        E.append(timestep.energy(disc, out["u_prev"], out["u"], dt))
    E = np.array(E)
    assert np.abs(E - E[0]).max() < 1e-11 * abs(E[0])


def test_energy_balance_with_ricker_load(c1):
    cfg, disc = c1
    dt = 0.9 * timestep.critical_dt(disc)
    ks = list(range(0, 121))
    out = timestep.cdm(disc, dt, 121, sources=cfg["sources"], checkpoints=ks)
    S = out["snapshots"]
    b = load_vector(disc, cfg["sources"][0])
    for k in (5, 40, 77, 119):
        e_plus = timestep.energy(disc, S[k], S[k + 1], dt)
        e_minus = timestep.energy(disc, S[k - 1], S[k], dt)
        Fk = problem.ricker(k * dt, 10.0) * b
        rhs = 0.5 * Fk @ (S[k + 1] - S[k - 1])
        assert abs((e_plus - e_minus) - rhs) < 1e-10 * max(abs(e_plus), 1e-30)


def test_reciprocity_and_linearity(c1):
    cfg, disc = c1
    prob = disc.prob
    dt = 0.9 * timestep.critical_dt(disc)
    A = dict(x=(0.1, 0.1), amp=1.0, f0=10.0)
    B = dict(x=(0.83, 0.27), amp=1.0, f0=10.0)
    # a receiver reads u at x: r(x) = N(x)^T u, i.e. the load vector / rho
    rA = load_vector(disc, A) / prob.rho
    rB = load_vector(disc, B) / prob.rho
    tAB = timestep.cdm(disc, dt, 300, sources=[A], receivers=rB[None])["trace"][:, 0]
    tBA = timestep.cdm(disc, dt, 300, sources=[B], receivers=rA[None])["trace"][:, 0]
    assert np.abs(tAB).max() > 0
    np.testing.assert_allclose(tAB, tBA, atol=1e-12 * np.abs(tAB).max())
    uA = timestep.cdm(disc, dt, 150, sources=[A])["u"]
    uB = timestep.cdm(disc, dt, 150, sources=[B])["u"]
    uAB = timestep.cdm(disc, dt, 150, sources=[A, B])["u"]
    np.testing.assert_allclose(uAB, uA + uB, atol=1e-13 * np.abs(uAB).max())


def test_stability_threshold(c1):
    _, disc = c1
    rng = np.random.default_rng(5)
    act = disc.mass > 0
    u0 = rng.standard_normal(disc.prob.ndof) * act
    dtc = timestep.critical_dt(disc)
    # with v0 = 0 every mode evolves as cos(k theta_j) below dt_crit, so the mass norm
    # never exceeds its initial value; just above dt_crit the top mode grows
    mnorm = lambda u: math.sqrt(u @ (disc.mass * u))
    stable = timestep.cdm(disc, 0.99 * dtc, 2000, u0=u0)["u"]
    unstable = timestep.cdm(disc, 1.01 * dtc, 400, u0=u0)["u"]
    assert mnorm(stable) <= mnorm(u0) * (1 + 1e-9)
    assert mnorm(unstable) > 1e6 * mnorm(u0)


def test_eps_stabilisation_increases_dt(c1):
    # Sec. 2.6: removing small mass eigenvalues of cut cells enlarges dt_crit
    cfg, disc = c1
    cfg0 = dict(cfg, eps=0.0)
    disc0 = build(Problem.from_config(cfg0))
    assert timestep.critical_dt(disc) > 1.2 * timestep.critical_dt(disc0)


def test_elastic_apply_K_matches_assembled():
    cfg = workloads.scaled_config(3, 4, 2, seed=9, ncomp=3, porosity=0.1, rmin=0.1, rmax=0.2)
    disc = build(Problem.from_config(cfg))
    assert len(disc.cut_cells) > 0
    K = assembled_K(disc)
    u = np.random.default_rng(1).standard_normal(disc.prob.ndof)
    np.testing.assert_allclose(apply_K(disc, u), K @ u, atol=1e-12)
    assert abs((K - K.T)).max() < 1e-12


def test_resumed_run_equals_one_run(c1):
    """Continuing a run from its returned state gives the run's own later steps, bit for
    bit (the resumed loop is the same recurrence on the same arrays)."""
    cfg, disc = c1
    dt = 0.9 * timestep.critical_dt(disc)
    src = cfg["sources"]
    whole = timestep.cdm(disc, dt, 300, sources=src, checkpoints=(200, 300))
    part = timestep.cdm(disc, dt, 120, sources=src)
    part = timestep.cdm(disc, dt, 200, sources=src, resume=part, checkpoints=(200,))
    assert np.array_equal(part["u"], whole["snapshots"][200])
    part = timestep.cdm(disc, dt, 300, sources=src, resume=part)
    assert part["k"] == 300
    assert np.array_equal(part["u"], whole["u"]) and np.array_equal(part["u_prev"], whole["u_prev"])
