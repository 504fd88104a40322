"""Pins of the oracle's rotated-cube geometry (Sec. 3.1, the paper's benchmark: a cube of
edge 0.3 turned by the Cardan angles 10/10/10 degrees inside a cube of edge 0.5):

* the numbers of degrees of freedom printed in Table timing_discretizations for the
  spectral cell discretisations (n_e cells per direction, degree p; the number in
  parentheses is the count of the chosen mesh): the nodes of every cell that is not
  entirely outside the physical cube.  Eleven of the fifteen (p, n_e) pairs are
  reproduced exactly; for the other four the paper drops a few more cells than an exact
  overlap test does (rule not stated), and the differences are pinned as named here;
* the box-cube predicates against brute force (point sampling) on random boxes, and the
  unrotated cube against the closed-form interval test;
* the tree rule's physical volume of all cut and uncut cells against the cube's volume;
* the rotation's order: T = R_z R_y R_x is the order that reproduces the table (the other
  orders tried reproduce none of the counts).
"""
import numpy as np
import pytest

import workloads
from oracle import geometry, problem, quadrature

# (p, n_e): DOF count of the table
TABLE = {(2, 28): 52353, (3, 13): 22816, (4, 9): 21109, (5, 7): 22706, (3, 18): 52375,
         (4, 12): 43065, (5, 9): 40176, (3, 20): 69391, (4, 15): 75085, (3, 19): 60472,
         (2, 31): 69083, (3, 14): 27793, (4, 10): 27233, (5, 11): 67086, (3, 31): 226108}
# counts an exact overlap test does not reproduce: our count minus the table's
NOT_REPRODUCED = {(2, 28): 36, (3, 13): 72, (2, 31): 24, (3, 31): 72}


def _active_nodes(cfg):
    prob = problem.Problem.from_config(cfg)
    cls = geometry.classify_cells(prob)
    table = prob.cell_node_table()
    mark = np.zeros(prob.nnodes, dtype=bool)
    mark[table[cls != geometry.OUT].ravel()] = True
    return int(mark.sum())


@pytest.mark.parametrize("p,n", sorted(TABLE))
def test_dof_counts_of_the_table(p, n):
    got = _active_nodes(workloads.rotated_cube(n, p))
    assert got - TABLE[(p, n)] == NOT_REPRODUCED.get((p, n), 0), (p, n, got)


def test_other_rotation_orders_do_not_reproduce_the_table():
    a = np.deg2rad(10.0)
    rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    ry = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
    rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    for T in (rx @ ry @ rz, rz @ rx @ rz):
        hits = 0
        for (p, n), dof in list(TABLE.items())[:6]:
            cfg = workloads.rotated_cube(n, p)
            cfg["cube"]["rot"] = T
            hits += _active_nodes(cfg) == dof
        assert hits == 0


def test_box_predicates_against_sampling():
    rng = np.random.default_rng(7)
    cfg = workloads.rotated_cube(10, 2)
    c = cfg["cube"]
    cube = (c["center"], c["half"], c["rot"])
    lo = rng.uniform(-0.25, 0.2, (400, 3))
    hi = lo + rng.uniform(0.005, 0.08, (400, 3))
    reach, sep = geometry.box_cube_relation(lo, hi, cube)
    assert sep.any() and (~sep).any() and reach.any() and (~reach).any()
    for i in range(len(lo)):
        pts = lo[i] + (hi[i] - lo[i]) * rng.random((3000, 3))
        out = geometry.outside_cube(pts, cube)
        if sep[i]:
            assert out.all(), i          # nothing of the box lies inside the cube
        if not reach[i]:
            assert not out.any(), i      # the box lies inside the cube
        if (~out).any():
            assert not sep[i], i         # a sampled point inside: not separated
        if out.any():
            assert reach[i], i           # a sampled point outside: it reaches outside


def test_unrotated_cube_is_the_interval_test():
    cfg = workloads.rotated_cube(12, 2, angles=(0.0, 0.0, 0.0))
    prob = problem.Problem.from_config(cfg)
    cls = geometry.classify_cells(prob).reshape(12, 12, 12)
    h = 0.5 / 12
    lo = -0.25 + h * np.arange(12)
    hi = lo + h
    inside = (lo >= -0.15) & (hi <= 0.15)
    outside = (hi <= -0.15) | (lo >= 0.15)
    for k in range(12):
        for j in range(12):
            for i in range(12):
                want = (geometry.OUT if (outside[i] or outside[j] or outside[k]) else
                        geometry.UNCUT if (inside[i] and inside[j] and inside[k]) else
                        geometry.CUT)
                assert cls[k, j, i] == want, (i, j, k)


@pytest.mark.parametrize("depth,tol", [(1, 2e-2), (3, 5e-3)])
def test_physical_volume_is_the_cube_volume(depth, tol):
    n, p = 6, 2
    cfg = workloads.rotated_cube(n, p, tree_depth=depth)
    prob = problem.Problem.from_config(cfg)
    cls = geometry.classify_cells(prob)
    vol = np.sum(cls == geometry.UNCUT) * prob.h ** 3
    for cell in np.flatnonzero(cls == geometry.CUT):
        lo = prob.cell_lo(cell)
        vol += quadrature.physical_volume(p, lo, lo + prob.h, prob.void_center, prob.void_radius,
                                          depth, prob.cube)
    assert abs(vol - 0.3 ** 3) <= tol * 0.3 ** 3
