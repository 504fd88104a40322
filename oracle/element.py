"""Element integrands on one Cartesian cell (paper Sec. 2.2, eq. weak_form_extended).

A cell is the box [x0, x0+h]^d, mapped from [-1,1]^d by x = x0 + (xi+1) h/2.  Shape
functions are tensor products of the GLL-Lagrange polynomials of degree p; local node
a = i0 + (p+1) i1 + (p+1)^2 i2 (x fastest).  Vector problems order the local DOFs
component-major: local dof = comp * (p+1)^d + a.

The scalar stiffness integrand is alpha rho c^2 grad N_i . grad N_j and the mass
integrand alpha rho N_i N_j (eq. weak_form_extended).  Linear elasticity (not in the
paper; textbook isotropic Hooke law) uses alpha B^T D B with Voigt strains.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import itertools

import numpy as np

from .basis import gl_points, gll_points, lagrange, lagrange_deriv


def local_multi_index(p, dim):
    """(n_s, dim) integer array: the tensor index (i0, i1, i2) of each local node."""
    rng = range(p + 1)
    idx = [t[::-1] for t in itertools.product(*([rng] * dim))]  # x fastest
    return np.array(idx, dtype=np.int64)


def shape_functions(p, dim, xi):
    """Tensor-product GLL-Lagrange shape functions at reference points.

    xi: (npts, dim) in [-1,1]^dim.  Returns N (npts, n_s) and dN (npts, dim, n_s),
    derivatives with respect to xi.
    """
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    nodes, _ = gll_points(p)
    vals = [lagrange(nodes, xi[:, a]) for a in range(dim)]
    ders = [lagrange_deriv(nodes, xi[:, a]) for a in range(dim)]
    mi = local_multi_index(p, dim)
    npts, ns = xi.shape[0], mi.shape[0]
    N = np.ones((npts, ns))
    dN = np.ones((npts, dim, ns))
    for a in range(dim):
        N *= vals[a][:, mi[:, a]]
        for b in range(dim):
            dN[:, b, :] *= (ders[a] if a == b else vals[a])[:, mi[:, a]]
    return N, dN


def box_rule(p, lo, hi):
    """Gauss-Legendre (p+1)^d rule on the physical box [lo, hi] (Sec. 2.2)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    dim = lo.size
    x1, w1 = gl_points(p + 1)
    mi = local_multi_index(p, dim)
    pts = np.empty((mi.shape[0], dim))
    wts = np.ones(mi.shape[0])
    for a in range(dim):
        half = 0.5 * (hi[a] - lo[a])
        pts[:, a] = lo[a] + (x1[mi[:, a]] + 1.0) * half
        wts *= w1[mi[:, a]] * half
    return pts, wts


def physical_shape(p, dim, cell_lo, h, pts):
    """Shape functions and physical gradients of the cell [cell_lo, cell_lo+h]^d."""
    xi = 2.0 * (np.asarray(pts) - np.asarray(cell_lo)) / h - 1.0
    N, dN = shape_functions(p, dim, xi)
    return N, dN * (2.0 / h)


def scalar_integrals(p, dim, cell_lo, h, pts, wts, alpha_vals, rho, c):
    """Scalar-wave element matrices from a point rule (eq. weak_form_extended):

    K_ij = sum_q w_q a_q rho c^2 grad N_i(x_q) . grad N_j(x_q)
    M_ij = sum_q w_q a_q rho N_i(x_q) N_j(x_q)
    """
    N, G = physical_shape(p, dim, cell_lo, h, pts)
    wa = np.asarray(wts) * np.asarray(alpha_vals)
    K = rho * c * c * np.tensordot(G * wa[:, None, None], G, axes=([0, 1], [0, 1]))
    M = rho * np.einsum("q,qi,qj->ij", wa, N, N)
    return K, M


def lame(E, nu):
    """Lame constants of isotropic linear elasticity."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def elasticity_D(E, nu):
    """6x6 Hooke matrix in Voigt order (xx, yy, zz, yz, xz, xy), engineering shears."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] = lam + 2.0 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    return D


def strain_displacement(G):
    """Voigt B matrices (npts, 6, 3 n_s) from physical gradients G (npts, 3, n_s)."""
    npts, _, ns = G.shape
    B = np.zeros((npts, 6, 3 * ns))
    ux, uy, uz = slice(0, ns), slice(ns, 2 * ns), slice(2 * ns, 3 * ns)
    B[:, 0, ux] = G[:, 0]
    B[:, 1, uy] = G[:, 1]
    B[:, 2, uz] = G[:, 2]
    B[:, 3, uy] = G[:, 2]
    B[:, 3, uz] = G[:, 1]
    B[:, 4, ux] = G[:, 2]
    B[:, 4, uz] = G[:, 0]
    B[:, 5, ux] = G[:, 1]
    B[:, 5, uy] = G[:, 0]
    return B


def elastic_integrals(p, cell_lo, h, pts, wts, alpha_vals, rho, E, nu):
    """3-D isotropic elasticity element matrices from a point rule:

    K = sum_q w_q a_q B_q^T D B_q;  M = rho sum_q w_q a_q N N^T on each component
    (block diagonal, component-major local DOFs).
    """
    N, G = physical_shape(p, 3, cell_lo, h, pts)
    B = strain_displacement(G)
    D = elasticity_D(E, nu)
    wa = np.asarray(wts) * np.asarray(alpha_vals)
    DB = np.einsum("st,qtj->qsj", D, B)
    K = np.tensordot(B * wa[:, None, None], DB, axes=([0, 1], [0, 1]))
    Ms = rho * np.einsum("q,qi,qj->ij", wa, N, N)
    M = np.kron(np.eye(3), Ms)
    return K, M


def element_integrals(prob, cell_lo, pts, wts, alpha_vals):
    """Stiffness and consistent mass of one cell of ``prob`` from a point rule."""
    if prob.ncomp == 1:
        return scalar_integrals(prob.p, prob.dim, cell_lo, prob.h, pts, wts, alpha_vals,
                                prob.rho, prob.c)
    return elastic_integrals(prob.p, cell_lo, prob.h, pts, wts, alpha_vals, prob.rho,
                             prob.E, prob.nu)


def gll_lumped_mass(p, dim, h, rho):
    """Diagonal mass of an uncut cell from GLL quadrature (Sec. 2.2, 2.4: nodal lumping):
    m_a = rho (h/2)^d prod_k w_{i_k(a)}."""
    _, w = gll_points(p)
    mi = local_multi_index(p, dim)
    m = np.full(mi.shape[0], rho * (0.5 * h) ** dim)
    for a in range(dim):
        m *= w[mi[:, a]]
    return m
