"""Pins of the oracle's Ricker pulse, point-load vector and IMEX block mass against what
the paper's formulas and the mathematics fix (no retyped oracle formula):

* Ricker wavelet (eq. source_time): the pulse peaks at 1 at the time shift t_s taken
  from the paper, vanishes where q^2 = 1/2, has its two minima -2 e^{-3/2} where
  q^2 = 3/2, and starts at f_t(0) = -47 e^{-24} (q(0)^2 = 24);
* point load b = rho amp N(x_s) (eq. weak_form_extended with a Dirac source): the
  GLL-Lagrange basis reproduces every polynomial of degree <= p per direction, so
  sum_i b_i f(x_i) = rho amp f(x_s) for all such f (which fixes every N_i(x_s)); the
  support is the nodes of one cell; a source on a cell face gives the same vector as
  one a hair inside either neighbour;
* block mass of the IMEX split (Sec. 2.5): the entries of diag(M^dd, M^cc) add up to
  rho times (volume of the uncut cells + physical volume of the cut cells + alpha times
  their void volume), the total mass of the indicator-weighted domain.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import basis, geometry, problem, quadrature
from oracle import imex as ox


# ---------------------------------------------------------------- Ricker (eq. source_time)

def _ts(f0):
    return 2.0 * math.sqrt(6.0) / (math.pi * f0)


@pytest.mark.parametrize("f0", [10.0, 6.0, 2.5])
def test_ricker_peak_at_time_shift(f0):
    ts = _ts(f0)
    assert problem.ricker(ts, f0) == pytest.approx(1.0, abs=1e-15)
    # the peak is the maximum: nearby times are lower
    for dt in (1e-4, 1e-3, 1e-2):
        assert problem.ricker(ts - dt / f0, f0) < 1.0
        assert problem.ricker(ts + dt / f0, f0) < 1.0


@pytest.mark.parametrize("f0", [10.0, 6.0])
def test_ricker_zeros_and_minima(f0):
    ts = _ts(f0)
    z = 1.0 / (math.sqrt(2.0) * math.pi * f0)  # q^2 = 1/2
    for t in (ts - z, ts + z):
        assert abs(problem.ricker(t, f0)) < 1e-14
    m = math.sqrt(1.5) / (math.pi * f0)  # q^2 = 3/2: minima of (1 - 2q^2) e^{-q^2}
    for t in (ts - m, ts + m):
        assert problem.ricker(t, f0) == pytest.approx(-2.0 * math.exp(-1.5), rel=1e-14)


def test_ricker_start_value():
    # q(0) = -pi f0 t_s = -2 sqrt(6): f_t(0) = (1 - 48) e^{-24}, independent of f0
    for f0 in (10.0, 3.0):
        assert problem.ricker(0.0, f0) == pytest.approx(-47.0 * math.exp(-24.0), rel=1e-12)


# ---------------------------------------------------------------- point load

def _node_coords(prob):
    """Coordinates of every node of the structured grid (per direction)."""
    xg, _ = basis.gll_points(prob.p)
    out = []
    for k in range(prob.dim):
        n = prob.ncells[k]
        x = np.empty(n * prob.p + 1)
        for cell in range(n):
            x[cell * prob.p: cell * prob.p + prob.p + 1] = (
                prob.lo[k] + cell * prob.h + 0.5 * (xg + 1.0) * prob.h)
        out.append(x)
    return out


def _grid_eval(prob, f):
    """f evaluated at every node (x fastest)."""
    xs = _node_coords(prob)
    mesh = np.meshgrid(*xs[::-1], indexing="ij")
    pts = [m.ravel() for m in mesh[::-1]]
    return f(*pts)


def _poly(rng, p, dim):
    """A random polynomial of degree <= p in each variable (tensor product)."""
    coef = rng.standard_normal((p + 1,) * dim)

    def f(*x):
        out = 0.0
        for idx in np.ndindex(*coef.shape):
            term = coef[idx]
            for k in range(dim):
                term = term * np.asarray(x[k], dtype=np.float64) ** idx[k]
            out = out + term
        return out
    return f


@pytest.mark.parametrize("dim,p,n", [(2, 3, 5), (2, 4, 4), (3, 2, 3)])
def test_load_reproduces_tensor_polynomials(dim, p, n):
    cfg = workloads._base(dim, (n,) * dim, p, np.zeros((0, dim)), np.zeros(0), rho=1.7)
    disc = problem.build(problem.Problem.from_config(cfg))
    prob = disc.prob
    rng = np.random.default_rng(11)
    for trial in range(4):
        xs = rng.uniform(0.02, 0.98, dim)
        amp = rng.uniform(0.5, 2.0)
        b = problem.load_vector(disc, dict(x=tuple(xs), amp=amp))
        # partition of unity and linear reproduction
        assert b.sum() == pytest.approx(prob.rho * amp, rel=1e-13)
        for k in range(dim):
            xk = _grid_eval(prob, lambda *x: x[k])
            assert b @ xk == pytest.approx(prob.rho * amp * xs[k], rel=1e-12)
        # every polynomial of degree <= p per direction
        f = _poly(rng, p, dim)
        assert b @ _grid_eval(prob, f) == pytest.approx(prob.rho * amp * f(*xs), rel=1e-10,
                                                        abs=1e-12)
        # support: the nodes of one cell
        nz = np.flatnonzero(b)
        cells = [c for c in range(disc.cell_nodes.shape[0])
                 if set(nz) <= set(disc.cell_nodes[c].tolist())]
        assert len(cells) >= 1


def test_load_on_cell_face_is_continuous():
    cfg = workloads._base(2, (4, 4), 3, np.zeros((0, 2)), np.zeros(0))
    disc = problem.build(problem.Problem.from_config(cfg))
    x_face = (0.5, 0.37)  # on the face between cells (1, 1) and (2, 1)
    b = problem.load_vector(disc, dict(x=x_face))
    for shift in (-1e-13, 1e-13):
        bs = problem.load_vector(disc, dict(x=(0.5 + shift, 0.37)))
        assert np.max(np.abs(bs - b)) < 1e-11


def test_load_elastic_direction():
    cfg = workloads._base(3, (3, 3, 3), 2, np.zeros((0, 3)), np.zeros(0), ncomp=3)
    disc = problem.build(problem.Problem.from_config(cfg))
    nn = disc.prob.nnodes
    d = np.array([0.3, -0.5, 0.8])
    b = problem.load_vector(disc, dict(x=(0.4, 0.55, 0.2), dir=tuple(d), amp=2.0))
    scalar = b[:nn] / d[0]
    for comp in range(3):
        assert np.allclose(b[comp * nn:(comp + 1) * nn], d[comp] * scalar, rtol=0, atol=1e-15)
    assert scalar.sum() == pytest.approx(2.0, rel=1e-13)


# ---------------------------------------------------------------- IMEX block mass (Sec. 2.5)

@pytest.mark.parametrize("dim,n,p,ncomp,alpha", [(2, 6, 2, 1, 1e-3), (2, 5, 3, 1, 0.2),
                                                 (3, 3, 2, 3, 1e-2)])
def test_block_mass_total_is_indicator_weighted_volume(dim, n, p, ncomp, alpha):
    if dim == 2:
        centers, radii = [(0.47, 0.52)], [0.23]
    else:
        centers, radii = [(0.5, 0.45, 0.55)], [0.31]
    cfg = workloads._base(dim, (n,) * dim, p, centers, radii, ncomp=ncomp, alpha=alpha,
                          rho=1.3)
    disc = problem.build(problem.Problem.from_config(cfg))
    prob = disc.prob
    c, d = ox.partition(disc)
    assert len(c) > 0 and len(d) > 0
    m_dd, Mcc = ox.mass_matrices(disc, c, d)
    total = m_dd.sum() + Mcc.sum()
    hd = prob.h ** dim
    vol = len(disc.uncut_cells) * hd
    for cell in disc.cut_cells:
        lo = prob.cell_lo(int(cell))
        vphys = quadrature.physical_volume(p, lo, lo + prob.h, prob.void_center,
                                           prob.void_radius, prob.tree_depth)
        vol += vphys + alpha * (hd - vphys)
    assert total == pytest.approx(ncomp * prob.rho * vol, rel=1e-13)
    # and the uncut cells alone: the diagonal of the explicit DOFs plus the uncut part of
    # M^cc is the GLL mass of those cells (their weights add up to the cell volume)
    assert np.all(m_dd > 0)
    assert geometry.UNCUT in set(disc.cls.tolist())
