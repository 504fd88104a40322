"""Sensitivity of the oracle's IMEX and consistent-mass results to rounding-sized changes
of the cut-cell matrices: the measurement that sets the parity bars of the device tests
of those schemes (Sec. 2.5 with the paper's alpha = 1e-12).

Two implementations of the tree quadrature (oracle and device) sum the same products in
different orders, so their cut-cell matrices differ by a few ulp.  A relative change of
1e-15 of every cut-cell stiffness and mass entry is applied here (symmetric, seeded) and
the state after 200 steps of the C1 problem is compared with the unperturbed one.  The
device tests must allow at least this much; they allow 10x more and fail above that:

* alpha = 1e-4 (cond(S) ~ 3e5): the change stays below 1e-12, bar 1e-10;
* alpha = 1e-12 (cond(S) ~ 6e12): IMEX moves by ~1e-6, bar 1e-5;
  consistent-mass central differences by ~1e-11, bar 1e-8.
"""
import copy

import numpy as np
import pytest

import workloads
from oracle import imex as ox
from oracle import problem, timestep

IMEX_BARS = {1e-4: 1e-10, 1e-12: 1e-5}
CONSISTENT_BARS = {1e-4: 1e-10, 1e-12: 1e-8}


def _perturbed(disc, rel, seed):
    rng = np.random.default_rng(seed)
    out = copy.copy(disc)

    def sym(shape):
        r = rng.uniform(-1.0, 1.0, shape)
        return 0.5 * (r + np.swapaxes(r, -1, -2))

    out.K_cut = disc.K_cut * (1.0 + rel * sym(disc.K_cut.shape))
    out.Mo_cut = disc.Mo_cut * (1.0 + rel * sym(disc.Mo_cut.shape))
    return out


def _c1(alpha):
    cfg = workloads.config("c1")
    cfg["alpha"] = alpha
    return cfg, problem.build(problem.Problem.from_config(cfg))


def _consistent_dt(disc):
    c, d = ox.partition(disc)
    m_dd, Mcc = ox.mass_matrices(disc, c, d)
    act = np.concatenate([d, c])
    n = len(act)
    M = np.zeros((n, n))
    M[:len(d), :len(d)] = np.diag(m_dd)
    M[len(d):, len(d):] = Mcc.toarray()
    K = problem.assembled_K(disc)[act][:, act].toarray()
    Li = np.linalg.inv(np.linalg.cholesky(M))
    return 0.9 * 2.0 / np.sqrt(np.linalg.eigvalsh(Li @ K @ Li.T)[-1])


@pytest.mark.parametrize("alpha", [1e-4, 1e-12])
def test_imex_sensitivity_sets_the_bar(alpha):
    cfg, disc = _c1(alpha)
    dt = 0.9 * timestep.critical_dt(disc)
    ref = ox.imex(disc, dt, 200, sources=cfg["sources"])["u"]
    worst = 0.0
    for seed in (1, 2):
        got = ox.imex(_perturbed(disc, 1e-15, seed), dt, 200, sources=cfg["sources"])["u"]
        worst = max(worst, np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"IMEX alpha={alpha:g}: relative change {worst:.2e} (bar {IMEX_BARS[alpha]:g})")
    assert worst <= IMEX_BARS[alpha] / 10
    if alpha == 1e-12:
        # ill-conditioned: a 1e-10 bar would reject a correct device result
        assert worst > 1e-9


@pytest.mark.parametrize("alpha", [1e-4, 1e-12])
def test_consistent_mass_sensitivity_sets_the_bar(alpha):
    cfg, disc = _c1(alpha)
    dt = _consistent_dt(disc)
    ref = ox.cdm_consistent(disc, dt, 200, sources=cfg["sources"])["u"]
    worst = 0.0
    for seed in (1, 2):
        pert = _perturbed(disc, 1e-15, seed)
        got = ox.cdm_consistent(pert, dt, 200, sources=cfg["sources"])["u"]
        worst = max(worst, np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"consistent alpha={alpha:g}: relative change {worst:.2e} "
          f"(bar {CONSISTENT_BARS[alpha]:g})")
    assert worst <= CONSISTENT_BARS[alpha] / 10
