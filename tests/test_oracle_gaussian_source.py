"""Pins of the oracle's volumetric Gaussian source (Sec. 3.1: f_s = exp(-|x - x_s|^2 /
(2 sigma^2)) times the Ricker pulse), from what the integral fixes:

* in an uncut box with the source far from every boundary, sum_i b_i = rho amp
  (2 pi)^{d/2} sigma^d (partition of unity), sum_i b_i x_i = x_s sum_i b_i (first moment,
  linear reproduction) and sum_i b_i (x_i - x_s)_k^2 = sigma^2 sum_i b_i (second moment,
  quadratic reproduction for p >= 2): a wrong width, centre or weight fails them;
* at the centre of a face of the rotated cube, about half of the Gaussian lies outside
  and is scaled by alpha;
* b vanishes outside the nodes of the cells within 8 sigma of x_s.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import problem


def _node_coords(prob):
    from oracle import basis
    xg = np.asarray(basis.gll_points(prob.p)[0])
    coords = []
    for k in range(prob.dim):
        c = np.empty(prob.ncells[k] * prob.p + 1)
        for e in range(prob.ncells[k]):
            lo = prob.lo[k] + e * prob.h
            c[e * prob.p:(e + 1) * prob.p + 1] = lo + 0.5 * prob.h * (xg + 1.0)
        coords.append(c)
    mesh = np.meshgrid(*coords[::-1], indexing="ij")
    return [m.ravel() for m in mesh[::-1]]


@pytest.mark.parametrize("dim,n,p,sigma", [(2, 12, 3, 0.03), (2, 10, 2, 0.05), (3, 8, 2, 0.04)])
def test_moments_in_an_uncut_box(dim, n, p, sigma):
    cfg = workloads._base(dim, (n,) * dim, p, np.zeros((0, dim)), np.zeros(0), rho=1.3)
    disc = problem.build(problem.Problem.from_config(cfg))
    prob = disc.prob
    xs = np.array([0.52, 0.47, 0.45][:dim])
    amp = 0.8
    b = problem.load_vector(disc, dict(x=tuple(xs), sigma=sigma, amp=amp))
    total = prob.rho * amp * (2.0 * math.pi) ** (dim / 2) * sigma ** dim
    assert b.sum() == pytest.approx(total, rel=1e-6)
    X = _node_coords(prob)
    for k in range(dim):
        assert b @ X[k] == pytest.approx(xs[k] * total, rel=1e-6)
        assert b @ (X[k] - xs[k]) ** 2 == pytest.approx(sigma ** 2 * total, rel=1e-5)
    # support: nodes of cells within 8 sigma of the source
    cells = problem.gaussian_support(prob, disc.cls, xs, sigma)
    allowed = np.zeros(prob.nnodes, dtype=bool)
    allowed[disc.cell_nodes[cells].ravel()] = True
    assert not np.any(b[~allowed])


def test_half_of_the_gaussian_outside_the_cube_face():
    cfg = workloads.rotated_cube(10, 3, tree_depth=2, alpha=1e-4)
    disc = problem.build(problem.Problem.from_config(cfg))
    sigma = 0.01
    src = dict(x=cfg["sources"][0]["x"], sigma=sigma, amp=1.0)
    b = problem.load_vector(disc, src)
    full = (2.0 * math.pi) ** 1.5 * sigma ** 3
    assert b.sum() == pytest.approx(0.5 * (1.0 + 1e-4) * full, rel=2e-2)
