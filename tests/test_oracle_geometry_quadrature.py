"""Pins of the oracle's classification, tree quadrature and stabilisation against
brute force, analytic areas/volumes and the identities of the paper's Sec. 2.6."""
import numpy as np
import pytest
from scipy import integrate

import workloads
from oracle import geometry, quadrature, stabilize
from oracle.problem import Problem, build, cut_cell_matrices, reference_element


def _prob(dim, n, p, centers, radii, depth=3, alpha=1e-12, ncomp=1, eps=1e-4):
    return Problem(dim=dim, ncomp=ncomp, ncells=(n,) * dim, lo=(0.0,) * dim, hi=(1.0,) * dim,
                   p=p, tree_depth=depth, void_center=np.asarray(centers, float),
                   void_radius=np.asarray(radii, float), alpha=alpha, eps=eps)


def test_classification_brute_force_sampling():
    cc, rr = workloads.random_circles(seed=7, count=12, rmin=0.03, rmax=0.12)
    prob = _prob(2, 12, 2, cc, rr)
    cls = geometry.classify_cells(prob)
    g = (np.arange(64) + 0.5) / 64
    checked = ncut = seen = 0
    for cell in range(prob.ncells[0] ** 2):
        lo = prob.cell_lo(cell)
        X, Y = np.meshgrid(lo[0] + g * prob.h, lo[1] + g * prob.h)
        pts = np.stack([X.ravel(), Y.ravel()], 1)
        inside = geometry.in_void(pts, cc, rr)
        # per-void containment by sampling
        contained = any(np.all(np.sum((pts - c) ** 2, 1) < r * r) for c, r in zip(cc, rr))
        if cls[cell] == geometry.UNCUT:
            assert not inside.any()
        elif cls[cell] == geometry.OUT:
            assert inside.all() and contained
        else:
            assert not contained
            ncut += 1
            seen += bool(inside.any())   # misses only thin slivers below the sampling
        checked += 1
    assert checked == 144
    assert ncut > 10 and seen >= 0.9 * ncut


def test_c1_counts_match_symmetry():
    # hole r = 1/4 at the centre of a 16x16 grid: cell classes are invariant under the
    # 8 symmetries of the square and the physical area of the cut cells plus the
    # uncut cells approximates 1 - pi/16
    cfg = workloads.config("c1")
    prob = Problem.from_config(cfg)
    cls = geometry.classify_cells(prob).reshape(16, 16)
    for t in (cls.T, cls[::-1], cls[:, ::-1], cls[::-1, ::-1]):
        np.testing.assert_array_equal(cls, t)
    assert (cls == geometry.UNCUT).sum() + (cls == geometry.CUT).sum() + (cls == geometry.OUT).sum() == 256


def _disc_box_area(lo, hi, c, r):
    """Area of box [lo,hi] inside the disc (c, r), integrating chord lengths."""
    def chord(x):
        s2 = r * r - (x - c[0]) ** 2
        if s2 <= 0:
            return 0.0
        s = np.sqrt(s2)
        return max(0.0, min(hi[1], c[1] + s) - max(lo[1], c[1] - s))
    x0, x1 = max(lo[0], c[0] - r), min(hi[0], c[0] + r)
    if x1 <= x0:
        return 0.0
    return integrate.quad(chord, x0, x1, epsabs=1e-15, epsrel=1e-13, limit=200)[0]


def _ball_box_volume(lo, hi, c, r):
    def area(z):
        s2 = r * r - (z - c[2]) ** 2
        if s2 <= 0:
            return 0.0
        return _disc_box_area(lo[:2], hi[:2], c[:2], np.sqrt(s2))
    z0, z1 = max(lo[2], c[2] - r), min(hi[2], c[2] + r)
    return integrate.quad(area, z0, z1, epsabs=1e-13, epsrel=1e-11, limit=200)[0]


@pytest.mark.parametrize("dim", [2, 3])
def test_tree_volume_converges_to_analytic(dim):
    # a single void cutting a unit-size cell; the physical volume seen by the tree
    # rule converges to the exact volume at first order in the leaf size
    c = np.array([0.83, 0.61, 0.47][:dim])
    r = 0.55
    lo, hi = np.zeros(dim), np.ones(dim)
    exact = 1.0 - (_disc_box_area(lo, hi, c, r) if dim == 2 else _ball_box_volume(lo, hi, c, r))
    errs = []
    for depth in ((2, 4, 6, 8) if dim == 2 else (2, 3, 4, 5)):
        vol = quadrature.physical_volume(2, lo, hi, c[None], [r], depth)
        errs.append(abs(vol - exact))
    assert errs[-1] < 2e-3 if dim == 2 else errs[-1] < 2e-2
    for a, b in zip(errs, errs[1:]):
        assert b < a


def test_tree_no_void_reproduces_reference():
    for dim, p, ncomp in [(2, 3, 1), (2, 4, 1), (3, 2, 3)]:
        prob = _prob(dim, 4, p, np.full((1, dim), 5.0), [0.1], ncomp=ncomp)
        K, Mo, av = cut_cell_matrices(prob, 5)
        Kr, Mf, _ = reference_element(prob)
        assert not av
        np.testing.assert_allclose(K, Kr, atol=1e-13 * np.abs(Kr).max())
        np.testing.assert_allclose(Mo, Mf, atol=1e-15)


def test_alpha_linearity_identity():
    # eq. alpha_stabilization: M(alpha) = M(0) + alpha (M^f - M(0)), same for K
    cc, rr = [[0.43, 0.58]], [0.31]
    for alpha in (1e-4, 0.25):
        p0 = _prob(2, 4, 3, cc, rr, alpha=0.0)
        pa = _prob(2, 4, 3, cc, rr, alpha=alpha)
        cell = 5
        assert geometry.classify_cells(p0)[cell] == geometry.CUT
        K0, M0, _ = cut_cell_matrices(p0, cell)
        Ka, Ma, _ = cut_cell_matrices(pa, cell)
        Kf, Mf, _ = reference_element(p0)
        np.testing.assert_allclose(Ma, M0 + alpha * (Mf - M0), atol=1e-15)
        np.testing.assert_allclose(Ka, K0 + alpha * (Kf - K0), atol=1e-12)


def test_mass_sum_is_physical_area_plus_alpha_void():
    cc, rr = [[0.43, 0.58]], [0.31]
    alpha = 1e-3
    prob = _prob(2, 4, 3, cc, rr, alpha=alpha, depth=5)
    cell = 5
    _, Mo, _ = cut_cell_matrices(prob, cell)
    lo = prob.cell_lo(cell)
    phys = quadrature.physical_volume(3, lo, lo + prob.h, np.array(cc), rr, 5)
    assert abs(Mo.sum() - (phys + alpha * (prob.h ** 2 - phys))) < 1e-14


def test_evs_identities():
    cfg = workloads.config("c1")
    prob = Problem.from_config(cfg)
    disc = build(prob)
    _, Mf, _ = reference_element(prob)
    seen_small = False
    for Mo in disc.Mo_cut:
        ms, margin, k = stabilize.evs_matrix(Mo, Mf, prob.f_lambda)
        if k == 0:
            assert np.all(ms == 0)
            continue
        seen_small = True
        # M~^s is an orthogonal projector of rank k: recover it by its trace scale
        t = np.trace(ms) / k
        P = ms / t
        np.testing.assert_allclose(P @ P, P, atol=1e-12)
        assert abs(np.trace(P) - k) < 1e-10
        assert abs(np.max(ms) - np.max(Mf)) < 1e-15 * np.max(Mf) * 10
        # the projector is orthogonal to the large-eigenvalue eigenvectors of M^o
        lam, phi = np.linalg.eigh(Mo)
        big = lam >= prob.f_lambda * lam[-1]
        assert np.abs(P @ phi[:, big]).max() < 1e-10
        assert margin > 1e-10
    assert seen_small
    # an uncut cell has no small eigenvalues at f_lambda = 1e-4
    _, _, k = stabilize.evs_matrix(Mf, Mf, prob.f_lambda)
    assert k == 0


def test_hrz_properties():
    cfg = workloads.config("c1")
    disc = build(Problem.from_config(cfg))
    for Mo, lump in zip(disc.Mo_cut, disc.lumped_cut):
        d = stabilize.hrz_diagonal(Mo, Mo.sum())
        assert np.all(d > 0)
        assert abs(d.sum() - Mo.sum()) < 1e-15 * 10
        assert np.all(lump >= d * (1 - 1e-14))   # eps diag(M^s) >= 0
    # eps = 0 leaves pure HRZ
    cfg["eps"] = 0.0
    disc0 = build(Problem.from_config(cfg))
    for Mo, lump in zip(disc0.Mo_cut, disc0.lumped_cut):
        np.testing.assert_allclose(lump, stabilize.hrz_diagonal(Mo, Mo.sum()), rtol=1e-15)
