"""1-D bases and quadrature rules (paper Sec. 2.2: GLL-Lagrange shape functions of the
spectral element / spectral cell method, GL quadrature in uncut and leaf cells).

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def gll_points(p):
    """Gauss-Lobatto-Legendre nodes and weights of order p (p+1 points) on [-1,1].

    Nodes: -1, +1 and the roots of P_p'.  Weights: w_i = 2 / (p(p+1) P_p(x_i)^2).
    These are the interpolation nodes of the SEM/SCM shape functions and the
    quadrature of the (diagonal) mass matrix in uncut cells (Sec. 2.2, Sec. 2.4).
    """
    if p < 1:
        raise ValueError("p >= 1")
    Pp = L.Legendre.basis(p)
    interior = np.sort(np.real(Pp.deriv().roots())) if p > 1 else np.zeros(0)
    x = np.concatenate(([-1.0], interior, [1.0]))
    w = 2.0 / (p * (p + 1) * Pp(x) ** 2)
    return x, w


def gl_points(n):
    """Gauss-Legendre rule with n points on [-1,1]; exact to degree 2n-1 (Sec. 2.2:
    p+1 points per direction in uncut cells and in every leaf of the space tree)."""
    x, w = L.leggauss(n)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def lagrange(nodes, x):
    """Values of the Lagrange polynomials on ``nodes`` at points ``x``.

    Returns an array of shape (len(x), len(nodes)):  l_i(x) = prod_{j!=i} (x-x_j)/(x_i-x_j).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                out[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return out


def lagrange_deriv(nodes, x):
    """Derivatives of the Lagrange polynomials on ``nodes`` at points ``x``.

    Product rule:  l_i'(x) = sum_{k!=i} 1/(x_i-x_k) prod_{j!=i,k} (x-x_j)/(x_i-x_j).
    Shape (len(x), len(nodes)).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for i in range(n):
        for k in range(n):
            if k == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[k]))
            for j in range(n):
                if j != i and j != k:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            out[:, i] += term
    return out
