"""Geometry of the immersed problem (paper Sec. 2.2): the physical domain is the
Cartesian box minus a union of balls (voids), optionally intersected with a rotated cube
(the benchmark geometry of Sec. 3.1: a cube of edge l_p turned by a rotation matrix T
about its centre inside the box); the fictitious part carries the indicator value alpha.

Exact FP64 predicates:
  * balls, on squared distances: a point is in a void iff |x - c|^2 < r^2 (points on a
    void's surface are physical), a box meets a void iff the squared distance from the
    centre to the box is < r^2, and a box lies inside a void iff the squared distance
    to its farthest corner is <= r^2;
  * the rotated cube (centre c, half edge a, axes u_j = columns of T), in local
    coordinates l_j = sum_k (x_k - c_k) T_kj: a point is outside iff |l_j| > a for some
    j (the cube's surface is physical); a box reaches outside iff one of its corners
    does (the cube is convex); a box lies outside (up to a zero-volume touch) iff an
    axis separates it from the cube: the box axes e_k, the cube axes u_j and, in 3-D,
    the products e_k x u_j (products shorter than 1e-10 are skipped); on axis L the
    test is |L.(b - c)| >= sum_k h_k |L_k| + a sum_j |L.u_j| with b, h the box centre
    and half edges.  Every sum is taken left to right in the index order written here.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np

OUT, UNCUT, CUT = 0, 1, 2


def cube_local(x, cube):
    """Local coordinates l (npts, d) of points x (npts, d) in the rotated cube's frame."""
    c, a, T = cube
    x = np.atleast_2d(x)
    d = x.shape[1]
    out = np.zeros_like(x, dtype=np.float64)
    for j in range(d):
        acc = (x[:, 0] - c[0]) * T[0][j]
        for k in range(1, d):
            acc = acc + (x[:, k] - c[k]) * T[k][j]
        out[:, j] = acc
    return out


def outside_cube(x, cube):
    """Boolean mask over points x: outside the (closed) rotated cube."""
    loc = cube_local(x, cube)
    return np.any(np.abs(loc) > cube[1], axis=1)


def in_void(x, centers, radii, cube=None):
    """Boolean mask over points x (npts, d): in the fictitious domain, i.e. inside some
    void (strict) or outside the rotated cube when there is one."""
    x = np.atleast_2d(x)
    hit = np.zeros(x.shape[0], dtype=bool)
    for c, r in zip(centers, radii):
        d2 = np.zeros(x.shape[0])
        for k in range(x.shape[1]):
            d2 = d2 + (x[:, k] - c[k]) * (x[:, k] - c[k])
        hit |= d2 < r * r
    if cube is not None:
        hit |= outside_cube(x, cube)
    return hit


def indicator(x, centers, radii, alpha, cube=None):
    """alpha^FCM(x): 1 in the physical domain, alpha in the fictitious part (Sec. 2.2)."""
    return np.where(in_void(x, centers, radii, cube), alpha, 1.0)


def _sat_axes(T, d):
    """Candidate separating axes of an axis-aligned box and the cube with axes T[:, j]."""
    axes = [tuple(1.0 if i == k else 0.0 for i in range(d)) for k in range(d)]
    axes += [tuple(T[i][j] for i in range(d)) for j in range(d)]
    if d == 3:
        for k in range(3):
            for j in range(3):
                u = (T[0][j], T[1][j], T[2][j])
                if k == 0:
                    L = (0.0, -u[2], u[1])
                elif k == 1:
                    L = (u[2], 0.0, -u[0])
                else:
                    L = (-u[1], u[0], 0.0)
                if (L[0] * L[0] + L[1] * L[1]) + L[2] * L[2] >= 1e-20:
                    axes.append(L)
    return axes


def box_cube_relation(lo, hi, cube):
    """(reaches_outside, outside) for boxes [lo, hi] (arrays (n, d) or (d,)) and the
    rotated cube: some corner outside the cube; an axis separates box and cube."""
    c, a, T = cube
    lo = np.atleast_2d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_2d(np.asarray(hi, dtype=np.float64))
    n, d = lo.shape
    reach = np.zeros(n, dtype=bool)
    for corner in np.ndindex(*(2,) * d):
        x = np.where(np.array(corner)[None, :] == 0, lo, hi)
        reach |= outside_cube(x, cube)
    sep = np.zeros(n, dtype=bool)
    for L in _sat_axes(T, d):
        dist = (0.5 * (lo[:, 0] + hi[:, 0]) - c[0]) * L[0]
        ra = (0.5 * (hi[:, 0] - lo[:, 0])) * abs(L[0])
        for k in range(1, d):
            dist = dist + (0.5 * (lo[:, k] + hi[:, k]) - c[k]) * L[k]
            ra = ra + (0.5 * (hi[:, k] - lo[:, k])) * abs(L[k])
        rb = 0.0
        for j in range(d):
            proj = T[0][j] * L[0]
            for k in range(1, d):
                proj = proj + T[k][j] * L[k]
            rb = rb + abs(proj)
        sep |= np.abs(dist) >= ra + a * rb
    return reach, sep


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


def box_status(lo, hi, centers, radii, cube=None):
    """OUT if the box lies inside one void or outside the cube, UNCUT if it meets no void
    and lies inside the cube, CUT otherwise."""
    meets_any = False
    if cube is not None:
        reach, sep = box_cube_relation(lo, hi, cube)
        if sep[0]:
            return OUT
        meets_any = bool(reach[0])
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
    cube = getattr(prob, "cube", None)
    if cube is not None:
        reach, sep = box_cube_relation(np.stack(lo, axis=1), np.stack(hi, axis=1), cube)
        meets |= reach
        contained |= sep
    cls = np.full(n, UNCUT, dtype=np.int8)
    cls[meets] = CUT
    cls[contained] = OUT
    return cls
