"""Pins of the oracle's observer rows (Sec. 3.2, observer traces) against what the
interpolation property of the GLL-Lagrange basis fixes: the row of a point x_r applied to
the nodal values of any tensor polynomial of degree <= p per direction gives the
polynomial's value at x_r (which fixes every N_a(x_r)); each row touches the nodes of one
cell and one component; a point on a cell face gives the row of a point a hair inside
either neighbour."""
import numpy as np
import pytest

import workloads
from oracle import problem


def _node_coords(disc):
    """Physical coordinates of every node (GLL points of each cell)."""
    from oracle import basis
    prob = disc.prob
    xg = np.asarray(basis.gll_points(prob.p)[0])
    coords = []
    for k in range(prob.dim):
        n = prob.ncells[k]
        c = np.empty(n * prob.p + 1)
        for e in range(n):
            lo = prob.lo[k] + e * prob.h
            c[e * prob.p:(e + 1) * prob.p + 1] = lo + 0.5 * prob.h * (xg + 1.0)
        coords.append(c)
    mesh = np.meshgrid(*coords[::-1], indexing="ij")
    return [m.ravel() for m in mesh[::-1]]


@pytest.mark.parametrize("dim,p,n,ncomp", [(2, 3, 5, 1), (2, 4, 3, 1), (3, 2, 3, 3), (3, 3, 2, 1)])
def test_rows_interpolate_tensor_polynomials(dim, p, n, ncomp):
    cfg = workloads._base(dim, (n,) * dim, p, np.zeros((0, dim)), np.zeros(0), ncomp=ncomp)
    disc = problem.build(problem.Problem.from_config(cfg))
    prob = disc.prob
    X = _node_coords(disc)
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.03, 0.97, (4, dim))
    R = problem.receiver_rows(disc, pts)
    assert R.shape == (4 * ncomp, prob.ndof)
    for trial in range(3):
        # a random tensor polynomial of degree <= p in each direction per component
        coef = rng.standard_normal((ncomp,) + (p + 1,) * dim)

        def f(comp, *x):
            v = 0.0
            for idx in np.ndindex(*(p + 1,) * dim):
                term = coef[(comp,) + idx]
                for k in range(dim):
                    term = term * x[k] ** idx[k]
                v = v + term
            return v

        u = np.concatenate([f(c, *X) for c in range(ncomp)])
        got = R @ u
        want = np.array([f(c, *x) for x in pts for c in range(ncomp)])
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-11 * np.abs(want).max())
    # support: the nodes of one cell, one component
    nn = prob.nnodes
    for row in range(R.shape[0]):
        nz = np.flatnonzero(R[row])
        comps = set((nz // nn).tolist())
        assert comps == {row % ncomp}
        nodes = set((nz % nn).tolist())
        assert any(nodes <= set(disc.cell_nodes[c].tolist()) for c in range(len(disc.cls)))


def test_row_on_cell_face_is_continuous():
    cfg = workloads._base(2, (4, 4), 3, np.zeros((0, 2)), np.zeros(0))
    disc = problem.build(problem.Problem.from_config(cfg))
    r = problem.receiver_rows(disc, [(0.25, 0.61)])
    for shift in (-1e-13, 1e-13):
        rs = problem.receiver_rows(disc, [(0.25 + shift, 0.61)])
        assert np.max(np.abs(rs - r)) < 1e-11
