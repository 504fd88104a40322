"""Pins of the IGA-FCM oracle (oracle/iga.py) against what the mathematics fixes: the
B-spline basis (partition of unity, reproduction of linear functions through the
Greville abscissae, the exact integral of every basis function, finite-difference
derivatives), the interior stencils of the uniform B-spline mass and stiffness in closed
form (autocorrelations of cardinal B-splines, Eulerian numbers), the closed-form row-sum
masses of a void-free box, the total mass with voids from the tree's physical volume, the
subspace relation K_IGA = A K_SCM A^T with the independently pinned SCM oracle (the
B-splines of a cell are polynomials of the SCM cell's space), the point load's moments
and the conservation of the discrete energy.  Each pin fails under a plausible mistake:
a dropped or misplaced recursion term, a wrong span, a transposed local order, a wrong
knot multiplicity, a mass summed over the wrong axis."""
import math

import numpy as np
import pytest

import workloads
from oracle import geometry, iga, quadrature
from oracle.basis import gl_points, gll_points
from oracle.problem import Problem, assembled_K, build as scm_build


def _prob(dim, n, p, centers=(), radii=(), depth=2, alpha=1e-3, rho=1.3, c=0.7):
    cc = np.asarray(centers, dtype=np.float64).reshape(-1, dim)
    cfg = workloads._base(dim, (n,) * dim, p, cc, np.asarray(radii, dtype=np.float64),
                          tree_depth=depth, alpha=alpha, rho=rho, c=c)
    return Problem.from_config(cfg)


def _greville(t, p):
    nb = len(t) - p - 1
    return np.array([t[i + 1:i + p + 1].mean() for i in range(nb)])


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_partition_of_unity_and_linear_reproduction(p):
    rng = np.random.default_rng(p)
    t = iga.knot_vector(7, p, -0.3, 0.25)
    x = np.concatenate([rng.uniform(t[0], t[-1], 200), t[p:-p]])  # knots included
    V = iga.bspline_values(t, p, x)
    assert V.shape == (len(x), 7 + p)
    assert V.min() >= -1e-15
    np.testing.assert_allclose(V.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(V @ _greville(t, p), x, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_integral_of_every_basis_function(p):
    """int N_i = (t_{i+p+1} - t_i) / (p + 1), integrated span by span with a GL rule of
    p + 1 points (exact for the degree-p pieces)."""
    h, n = 0.2, 9
    t = iga.knot_vector(n, p, 1.0, h)
    xg, wg = gl_points(p + 1)
    tot = np.zeros(n + p)
    for c in range(n):
        a = 1.0 + c * h
        x = a + 0.5 * h * (xg + 1.0)
        tot += (0.5 * h * wg) @ iga.bspline_values(t, p, x)
    exact = np.array([(t[i + p + 1] - t[i]) / (p + 1) for i in range(n + p)])
    np.testing.assert_allclose(tot, exact, rtol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_derivatives_against_central_differences(p):
    rng = np.random.default_rng(10 + p)
    t = iga.knot_vector(6, p, 0.0, 1.0)
    # points at least 1e-3 away from every knot (the pieces are polynomials there)
    x = rng.uniform(0.0, 6.0, 300)
    x = x[np.min(np.abs(x[:, None] - np.arange(7)[None, :]), axis=1) > 1e-3]
    eps = 1e-6
    fd = (iga.bspline_values(t, p, x + eps) - iga.bspline_values(t, p, x - eps)) / (2 * eps)
    np.testing.assert_allclose(iga.bspline_derivatives(t, p, x), fd, atol=2e-8)


def test_uniform_quadratic_closed_form():
    """The uniform quadratic B-spline on knots 0, 1, 2, 3: x^2/2, (-2x^2 + 6x - 3)/2,
    (3 - x)^2/2 on the three spans (the interior function of a long knot vector)."""
    t = iga.knot_vector(8, 2, -2.0, 1.0)  # knots -2 (x3), -1, 0, ..., 6 (x3)
    x = np.linspace(0.0, 3.0, 31)
    i = 4  # N_4 has the knots 0, 1, 2, 3
    assert np.allclose(t[i:i + 4], [0, 1, 2, 3])
    ref = np.where(x < 1, x * x / 2, np.where(x < 2, (-2 * x * x + 6 * x - 3) / 2, (3 - x) ** 2 / 2))
    np.testing.assert_allclose(iga.bspline_values(t, 2, x)[:, i], ref, atol=1e-14)


def _eulerian(n, k):
    return sum((-1) ** j * math.comb(n + 1, j) * (k + 1 - j) ** n for j in range(k + 1))


def _cardinal(m, j):
    """Cardinal B-spline of degree m (support [0, m + 1]) at the integer j:
    A(m, j - 1) / m! with the Eulerian numbers A."""
    if j < 1 or j > m:
        return 0.0
    return _eulerian(m, j - 1) / math.factorial(m)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_interior_stencils_closed_form(p):
    """Away from the box's faces the 1-D B-spline Gram matrices are Toeplitz:
    int N_a N_{a+k} = h B_{2p+1}(p + 1 + k) and int N_a' N_{a+k}' = -h^{-1} B''_{2p+1}(p + 1
    + k) with B''_m(x) = B_{m-2}(x) - 2 B_{m-2}(x - 1) + B_{m-2}(x - 2) (autocorrelation of
    the cardinal B-spline); in 2-D M = rho M1 (x) M1 and K = rho c^2 (K1 (x) M1 + M1 (x) K1)."""
    n = 3 * p + 3
    pr = _prob(2, n, p)
    d = iga.build(pr)
    K, M = iga.assembled(d)
    h = pr.h
    m1 = {k: h * _cardinal(2 * p + 1, p + 1 + k) for k in range(-p, p + 1)}
    s1 = {k: -(_cardinal(2 * p - 1, p + 1 + k) - 2 * _cardinal(2 * p - 1, p + k)
               + _cardinal(2 * p - 1, p - 1 + k)) / h for k in range(-p, p + 1)}
    assert abs(sum(s1.values())) < 1e-12 and abs(sum(m1.values()) - h) < 1e-14
    nb = n + p
    for a in range(2 * p, n - p):
        for b in range(2 * p, n - p):
            i = a + nb * b
            for k in range(-p, p + 1):
                for l in range(-p, p + 1):
                    j = (a + k) + nb * (b + l)
                    assert M[i, j] == pytest.approx(pr.rho * m1[k] * m1[l], rel=1e-12, abs=1e-15)
                    kk = pr.rho * pr.c ** 2 * (s1[k] * m1[l] + m1[k] * s1[l])
                    assert K[i, j] == pytest.approx(kk, rel=1e-11, abs=1e-13)
            # nothing beyond the stencil
            row = K[i].reshape(nb, nb)
            mask = np.ones_like(row, dtype=bool)
            mask[b - p:b + p + 1, a - p:a + p + 1] = False
            assert np.abs(row[mask]).max() == 0.0


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 4), (3, 2)])
def test_row_sum_mass_of_void_free_box(dim, p):
    """m_i = rho prod_k (t_{i_k+p+1} - t_{i_k}) / (p + 1)."""
    n = 5 if dim == 3 else 7
    pr = _prob(dim, n, p)
    d = iga.build(pr)
    t = iga.knot_vector(n, p, 0.0, pr.h)
    w1 = np.array([(t[i + p + 1] - t[i]) / (p + 1) for i in range(n + p)])
    ref = w1.copy()
    for _ in range(dim - 1):
        ref = np.multiply.outer(w1, ref).ravel()
    np.testing.assert_allclose(d.mass, pr.rho * ref, rtol=1e-13)
    K, _ = iga.assembled(d)
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-12)  # constants in the kernel


def test_total_mass_with_voids_and_dropped_cells():
    """sum_i m_i = rho (V of uncut cells + sum over kept cut cells of (V_phys + alpha
    V_void)) with V_phys from the tree (quadrature.physical_volume); a void swallowing a
    whole cell drops it, and the functions supported only there carry no mass."""
    cc = [(0.31, 0.52), (0.75, 0.2)]
    rr = [0.17, 0.08]
    pr = _prob(2, 10, 3, cc, rr, depth=3, alpha=1e-4)
    d = iga.build(pr)
    cls = d.cls
    assert (cls == geometry.OUT).any() and (cls == geometry.CUT).any()
    vol = pr.h ** 2 * np.count_nonzero(cls == geometry.UNCUT)
    for cell in np.flatnonzero(cls == geometry.CUT):
        lo = pr.cell_lo(int(cell))
        vp = quadrature.physical_volume(pr.p, lo, lo + pr.h, pr.void_center, pr.void_radius,
                                        pr.tree_depth)
        vol += vp + pr.alpha * (pr.h ** 2 - vp)
    assert d.mass.sum() == pytest.approx(pr.rho * vol, rel=1e-12)
    assert d.mass.min() >= 0.0
    # every DOF with mass is supported by a kept cell, every other one by none
    supported = np.zeros(d.ndof, dtype=bool)
    supported[d.cell_dofs[d.cells].ravel()] = True
    assert np.array_equal(supported, d.mass > 0)
    K, _ = iga.assembled(d)
    np.testing.assert_allclose(K @ np.ones(d.ndof), 0.0, atol=1e-11)


@pytest.mark.parametrize("dim,n,p", [(2, 6, 2), (2, 5, 3), (3, 4, 2)])
def test_stiffness_is_the_scm_stiffness_on_the_spline_subspace(dim, n, p):
    """The B-splines of degree p are polynomials of degree p per direction on every cell,
    so the spline space is a subspace of the SCM's continuous Lagrange space on the same
    cells: N_i = sum_j N_i(x_j) L_j with x_j the SCM nodes.  With the same quadrature
    (GL in uncut cells, the same tree in cut cells) K_IGA = A K_SCM A^T, A_ij = N_i(x_j),
    K_SCM from the SCM oracle."""
    if dim == 2:
        cc, rr = [(0.4, 0.45), (0.9, 0.1)], [0.21, 0.12]
    else:
        cc, rr = [(0.45, 0.5, 0.4)], [0.3]
    pr = _prob(dim, n, p, cc, rr, depth=2, alpha=1e-3)
    d = iga.build(pr)
    scm = scm_build(pr)
    assert np.array_equal(d.cls, scm.cls)
    Ks = assembled_K(scm).toarray()
    xi, _ = gll_points(p)
    t = iga.knot_vector(n, p, 0.0, pr.h)
    npn = n * p + 1
    xs = np.array([min(m // p, n - 1) * pr.h + 0.5 * pr.h * (xi[m - min(m // p, n - 1) * p] + 1.0)
                   for m in range(npn)])
    A1 = iga.bspline_values(t, p, xs).T  # (n + p, npn)
    A = A1
    for _ in range(dim - 1):
        A = np.kron(A1, A)
    K, _ = iga.assembled(d)
    ref = A @ Ks @ A.T
    np.testing.assert_allclose(K, ref, atol=1e-11 * np.abs(ref).max())


def test_point_load_moments():
    """sum_i b_i = rho amp (partition of unity); sum_i b_i g_i = rho amp x_s per direction
    (Greville reproduction); a source on a cell face gives the same b from either cell."""
    pr = _prob(2, 8, 3, [(0.8, 0.8)], [0.05])
    d = iga.build(pr)
    t = iga.knot_vector(8, 3, 0.0, pr.h)
    g = _greville(t, 3)
    nb = 11
    gx = np.tile(g, nb)
    gy = np.repeat(g, nb)
    for x in [(0.33, 0.41), (0.25, 0.6)]:  # the second lies on the face x = 2h
        b = iga.load_vector(d, dict(x=x, amp=2.5))
        assert b.sum() == pytest.approx(pr.rho * 2.5, rel=1e-14)
        assert b @ gx == pytest.approx(pr.rho * 2.5 * x[0], rel=1e-13)
        assert b @ gy == pytest.approx(pr.rho * 2.5 * x[1], rel=1e-13)
    # the face point taken in the cell on the left of the face
    _, N = iga.source_values(pr, (0.25, 0.6))
    kv = iga.knots(pr)
    left = 1 + 8 * 4  # cell (1, 4), whose upper x face is x = 0.25
    Nl, _ = iga.cell_shape(pr, kv, left, np.array([[0.25, 0.6]]))
    b1 = np.zeros(d.ndof)
    np.add.at(b1, d.cell_dofs[left], Nl[0])
    b2 = np.zeros(d.ndof)
    np.add.at(b2, d.cell_dofs[2 + 8 * 4], N)
    np.testing.assert_allclose(b1, b2, atol=1e-15)


def test_energy_conserved_without_load():
    """eq. cdm with the lumped IGA mass conserves 1/2 v^T M v + 1/2 u_{k+1}^T K u_k."""
    pr = _prob(2, 9, 3, [(0.5, 0.45)], [0.2], depth=2, alpha=1e-2)
    d = iga.build(pr)
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal(d.ndof) * (d.mass > 0)
    dt = 0.8 * iga.critical_dt(d)
    r = iga.cdm(d, dt, 60, u0=u0)
    E = [iga.energy(d, r["u_prev"], r["u"], dt)]
    r2 = iga.cdm(d, dt, 120, u0=u0)
    E.append(iga.energy(d, r2["u_prev"], r2["u"], dt))
    assert E[1] == pytest.approx(E[0], rel=1e-10)


def test_lumped_critical_step_does_not_collapse_on_small_cuts():
    """Row-sum lumping keeps the critical step of cut cells near that of the uncut mesh
    (Sec. 2.4; the lumped IGA-FCM step is the largest of the methods compared): a void
    that leaves tiny slivers of physical domain in its cut cells barely moves it."""
    pr0 = _prob(2, 8, 2, alpha=1e-8)
    pr1 = _prob(2, 8, 2, [(0.5, 0.5)], [0.2499], depth=3, alpha=1e-8)
    dt0 = iga.critical_dt(iga.build(pr0))
    dt1 = iga.critical_dt(iga.build(pr1))
    assert dt1 > 0.5 * dt0
