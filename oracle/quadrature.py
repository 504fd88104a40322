"""Space-tree (quadtree / octree) quadrature of cut cells (paper Sec. 1 and Sec. 2.2:
cut cells are integrated by recursive partitioning with Gauss-Legendre points in every
leaf, for all system matrices).

Reading of the paper (it gives no depth and no refinement rule): a box of the tree at
level l is
  * inside one void            -> integrated with the constant alpha,
  * free of every void         -> integrated with the constant 1,
  * otherwise, if l < depth    -> split into 2^d equal children,
  * otherwise (a leaf at depth) -> GL (p+1)^d points with the pointwise indicator.
Every box is integrated with the (p+1)^d Gauss-Legendre rule on that box; the
integrands of uncut sub-boxes are polynomials of degree <= 2p per direction, so that
rule is exact there.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import itertools

import numpy as np

from .element import box_rule
from .geometry import OUT, UNCUT, box_status, box_void_relation, indicator


def tree_boxes(lo, hi, centers, radii, depth, level=0, cube=None):
    """List of (lo, hi, kind) integration boxes of the space tree over [lo, hi].

    kind is 'alpha' (constant alpha), 'one' (constant 1) or 'leaf' (pointwise).
    """
    st = box_status(lo, hi, centers, radii, cube)
    if st == OUT:
        return [(lo, hi, "alpha")]
    if st == UNCUT:
        return [(lo, hi, "one")]
    if level >= depth:
        return [(lo, hi, "leaf")]
    mid = 0.5 * (lo + hi)
    out = []
    for corner in itertools.product((0, 1), repeat=len(lo)):
        c = np.array(corner)
        clo = np.where(c == 0, lo, mid)
        chi = np.where(c == 0, mid, hi)
        out.extend(tree_boxes(clo, chi, centers, radii, depth, level + 1, cube))
    return out


def tree_rule(p, lo, hi, centers, radii, alpha, depth, cube=None):
    """Quadrature points, weights and indicator values over one cut cell.

    Returns (pts, wts, alpha_vals, all_void) where all_void is True when every box of
    the tree lies inside a void (the cell is then dropped as being outside the
    physical domain).
    """
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    # a void that does not meet the cell meets none of its sub-boxes and contains none
    # of its points: keep only the voids meeting the cell (same predicates, fewer tests)
    keep = [j for j in range(len(radii)) if box_void_relation(lo, hi, centers[j], radii[j])[0]]
    centers = np.asarray(centers, float).reshape(len(radii), len(lo))[keep]
    radii = np.asarray(radii, float)[keep]
    boxes = tree_boxes(lo, hi, centers, radii, depth, cube=cube)
    P, W, A = [], [], []
    for blo, bhi, kind in boxes:
        pts, wts = box_rule(p, blo, bhi)
        if kind == "alpha":
            av = np.full(len(wts), alpha)
        elif kind == "one":
            av = np.ones(len(wts))
        else:
            av = indicator(pts, centers, radii, alpha, cube)
        P.append(pts)
        W.append(wts)
        A.append(av)
    all_void = all(kind == "alpha" for _, _, kind in boxes)
    return np.concatenate(P), np.concatenate(W), np.concatenate(A), all_void


def physical_volume(p, lo, hi, centers, radii, depth, cube=None):
    """Volume of the physical part of [lo,hi] as seen by the tree rule (alpha = 0)."""
    pts, wts, av, _ = tree_rule(p, lo, hi, centers, radii, 0.0, depth, cube)
    return float(np.sum(wts * av))
