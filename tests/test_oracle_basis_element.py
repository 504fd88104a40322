"""Pins of the oracle's bases and element matrices against textbook values and closed
forms (none of them re-derives the oracle's own formulas)."""
import math

import numpy as np
import pytest

from oracle import basis, element
from oracle.problem import Problem, reference_element

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def load_gll_table():
    """Textbook GLL nodes/weights (tests/golden/gll_textbook.txt)."""
    rows = {}
    with open(f"{GOLDEN}/gll_textbook.txt") as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            p, x, w = line.split()
            rows.setdefault(int(p), []).append((eval(x, {"sqrt": math.sqrt}),
                                                eval(w, {"sqrt": math.sqrt})))
    return rows


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_gll_textbook(p):
    table = load_gll_table()[p]
    x, w = basis.gll_points(p)
    ref = sorted(table)
    np.testing.assert_allclose(x, [r[0] for r in ref], atol=1e-14)
    np.testing.assert_allclose(w, [r[1] for r in ref], atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gl_exactness(n):
    x, w = basis.gl_points(n)
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - exact) < 1e-13
    k = 2 * n  # first degree not integrated exactly
    assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_lagrange_cardinal_and_derivative(p):
    nodes, _ = basis.gll_points(p)
    V = basis.lagrange(nodes, nodes)
    np.testing.assert_allclose(V, np.eye(p + 1), atol=1e-13)
    xs = np.linspace(-0.97, 0.97, 11)
    np.testing.assert_allclose(basis.lagrange(nodes, xs).sum(1), 1.0, atol=1e-13)
    hstep = 1e-6
    fd = (basis.lagrange(nodes, xs + hstep) - basis.lagrange(nodes, xs - hstep)) / (2 * hstep)
    np.testing.assert_allclose(basis.lagrange_deriv(nodes, xs), fd, atol=1e-6)
    # the interpolant of a polynomial of degree <= p is exact
    f = lambda t: 0.3 * t ** p - t + 0.25
    np.testing.assert_allclose(basis.lagrange(nodes, xs) @ f(nodes), f(xs), atol=1e-12)


def _prob(dim, p, h=0.5, ncomp=1, E=1.0, nu=0.3, rho=1.0, c=1.0):
    return Problem(dim=dim, ncomp=ncomp, ncells=(1,) * dim, lo=(0.0,) * dim, hi=(h,) * dim,
                   p=p, tree_depth=0, void_center=np.zeros((0, dim)), void_radius=np.zeros(0),
                   rho=rho, c=c, E=E, nu=nu)


def test_q1_square_laplace_textbook():
    # bilinear square element, Laplace operator: diag 2/3, edge neighbours -1/6,
    # opposite corner -1/3, independent of h (local order (0,0),(1,0),(0,1),(1,1))
    for h in (0.5, 0.125):
        K, Mf, lm = reference_element(_prob(2, 1, h=h, rho=2.0, c=1.5))
        ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
        np.testing.assert_allclose(K, 2.0 * 1.5 ** 2 * ref, atol=1e-14)
        # consistent mass of the bilinear square: rho h^2/36 [4 2 2 1; ...]
        mref = np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]]) / 36.0
        np.testing.assert_allclose(Mf, 2.0 * h * h * mref, atol=1e-15)
        np.testing.assert_allclose(lm, 2.0 * h * h / 4.0, atol=1e-15)


def test_q1_brick_laplace_textbook():
    # trilinear cube: diag h/3, edge neighbours 0, face diagonals -h/12, body diagonal -h/12
    h = 0.25
    K, _, _ = reference_element(_prob(3, 1, h=h))
    mi = element.local_multi_index(1, 3)
    for i in range(8):
        for j in range(8):
            nd = int(np.sum(mi[i] != mi[j]))
            ref = {0: h / 3, 1: 0.0, 2: -h / 12, 3: -h / 12}[nd]
            assert abs(K[i, j] - ref) < 1e-15


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_reference_scalar_invariants(dim, p):
    h = 0.37
    K, Mf, lm = reference_element(_prob(dim, p, h=h, rho=1.3))
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    assert np.abs(K @ np.ones(len(K))).max() < 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-12 * ev[-1]
    assert np.sum(ev < 1e-10 * ev[-1]) == 1
    assert abs(Mf.sum() - 1.3 * h ** dim) < 1e-14
    assert abs(lm.sum() - 1.3 * h ** dim) < 1e-14
    # GLL weights are the nodal lumping of the consistent mass only up to p: both
    # integrate a constant exactly; and GLL lumping is positive
    assert np.all(lm > 0)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_reference_elastic_energy_closed_forms(p):
    E, nu, h = 2.0, 0.3, 0.4
    prob = _prob(3, p, h=h, ncomp=3, E=E, nu=nu)
    K, _, _ = reference_element(prob)
    lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    ns = (p + 1) ** 3
    nodes, _ = basis.gll_points(p)
    mi = element.local_multi_index(p, 3)
    X = (nodes[mi] + 1.0) * h / 2  # (ns, 3) physical node coordinates
    eps0, gam = 1e-2, 3e-2
    u = np.zeros(3 * ns)
    u[:ns] = eps0 * X[:, 0]                      # uniaxial strain e_xx = eps0
    assert abs(u @ K @ u - (lam + 2 * mu) * eps0 ** 2 * h ** 3) < 1e-13
    u = np.zeros(3 * ns)
    u[:ns] = gam * X[:, 1]                       # engineering shear gamma_xy
    assert abs(u @ K @ u - mu * gam ** 2 * h ** 3) < 1e-13
    u = np.zeros(3 * ns)                         # hydrostatic strain
    u[:ns], u[ns:2 * ns], u[2 * ns:] = eps0 * X[:, 0], eps0 * X[:, 1], eps0 * X[:, 2]
    bulk = lam + 2 * mu / 3
    assert abs(u @ K @ u - 9 * bulk * eps0 ** 2 * h ** 3) < 1e-13
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev[-1]) == 6      # rigid body modes
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()


def test_elastic_nu0_decouples_like_scalar():
    # with nu = 0 (lambda = 0, mu = E/2) the x-x block of K equals mu (grad.grad + dx dx)
    prob = _prob(3, 2, h=0.3, ncomp=3, E=2.0, nu=0.0)
    K, _, _ = reference_element(prob)
    ks, _, _ = reference_element(_prob(3, 2, h=0.3))
    ns = 27
    off = K[:ns, ns:]
    # an x-displacement depending on y only is pure shear, energy mu*|grad u|^2
    nodes, _ = basis.gll_points(2)
    mi = element.local_multi_index(2, 3)
    X = (nodes[mi] + 1.0) * 0.15
    f = np.sin(2.0 * X[:, 1])
    assert abs(f @ K[:ns, :ns] @ f - 1.0 * (f @ ks @ f)) < 1e-12
    assert np.abs(off).max() > 0
