"""Geometry of the immersed problem (paper Sec. 2.2): the physical domain is the
Cartesian box minus a union of balls (voids); the fictitious part carries the
indicator value alpha.

Exact FP64 predicates on squared distances: a point is in a void iff
|x - c|^2 < r^2 (points on a void's surface are physical), a box meets a void iff
the squared distance from the centre to the box is < r^2, and a box lies inside a
void iff the squared distance to its farthest corner is <= r^2.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np

OUT, UNCUT, CUT = 0, 1, 2


def in_void(x, centers, radii):
    """Boolean mask over points x (npts, d): inside some void (strict)."""
    x = np.atleast_2d(x)
    hit = np.zeros(x.shape[0], dtype=bool)
    for c, r in zip(centers, radii):
        d2 = np.zeros(x.shape[0])
        for k in range(x.shape[1]):
            d2 = d2 + (x[:, k] - c[k]) * (x[:, k] - c[k])
        hit |= d2 < r * r
    return hit


def indicator(x, centers, radii, alpha):
    """alpha^FCM(x): 1 in the physical domain, alpha in the voids (Sec. 2.2)."""
    return np.where(in_void(x, centers, radii), alpha, 1.0)


def box_void_relation(lo, hi, c, r):
    """(meets, contained) for the box [lo,hi] and the ball (c, r)."""
    dmin2 = 0.0
    dmax2 = 0.0
    for k in range(len(lo)):
        gap = max(lo[k] - c[k], 0.0, c[k] - hi[k])
        far = max(abs(c[k] - lo[k]), abs(hi[k] - c[k]))
        dmin2 = dmin2 + gap * gap
        dmax2 = dmax2 + far * far
    return dmin2 < r * r, dmax2 <= r * r


def box_status(lo, hi, centers, radii):
    """OUT if the box lies inside one void, UNCUT if it meets none, CUT otherwise."""
    meets_any = False
    for c, r in zip(centers, radii):
        meets, contained = box_void_relation(lo, hi, c, r)
        if contained:
            return OUT
        meets_any |= meets
    return CUT if meets_any else UNCUT


def classify_cells(prob):
    """Class of every cell of the grid (paper Sec. 2.2 and Sec. 3.2.2: cells that lie
    entirely outside the physical domain are disregarded).  Vectorised over cells,
    same predicates as ``box_status``.  Returns int8 array in lexicographic cell
    order (x fastest)."""
    dim = prob.dim
    ncell = prob.ncells
    grids = np.meshgrid(*[np.arange(n) for n in ncell[::-1]], indexing="ij")
    idx = [g.ravel() for g in grids[::-1]]  # idx[0] = cx (fastest)
    lo = [prob.lo[k] + idx[k] * prob.h for k in range(dim)]
    hi = [prob.lo[k] + (idx[k] + 1) * prob.h for k in range(dim)]
    n = lo[0].size
    meets = np.zeros(n, dtype=bool)
    contained = np.zeros(n, dtype=bool)
    for c, r in zip(prob.void_center, prob.void_radius):
        dmin2 = np.zeros(n)
        dmax2 = np.zeros(n)
        for k in range(dim):
            gap = np.maximum(np.maximum(lo[k] - c[k], 0.0), c[k] - hi[k])
            far = np.maximum(np.abs(c[k] - lo[k]), np.abs(hi[k] - c[k]))
            dmin2 = dmin2 + gap * gap
            dmax2 = dmax2 + far * far
        meets |= dmin2 < r * r
        contained |= dmax2 <= r * r
    cls = np.full(n, UNCUT, dtype=np.int8)
    cls[meets] = CUT
    cls[contained] = OUT
    return cls
