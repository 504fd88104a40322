"""Assembly of the discrete immersed problem M u'' + K u = F (paper eq. semi).

Global DOFs live on the full structured node grid of the Cartesian mesh:
node = ix + nx (iy + ny iz) with n_k = ncells_k p + 1, and a vector problem stores
its components one after another (dof = comp * nnodes + node).  Nodes that belong to
no active cell carry no mass and stay zero.

Mass: GLL (nodal) lumping in uncut cells (Sec. 2.2, 2.4) and the stabilised HRZ
diagonal in cut cells (see ``stabilize``); assembled by summing element diagonals.
Stiffness: the uncut reference matrix (GL (p+1)^d rule, exact on a Cartesian cell) and
one tree-integrated matrix per cut cell.

Load: a point source f(x,t) = f_t(t) * amp * dir * delta(x - x_s) gives
F_i = rho * amp * dir_c * N_i(x_s) (eq. weak_form_extended with alpha(x_s) = 1) in a
cell containing x_s; the shape functions are continuous, so any such cell gives the
same vector.  f_t is the Ricker wavelet, eq. source_time.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import basis, element, geometry, quadrature, stabilize


@dataclass
class Problem:
    dim: int
    ncomp: int
    ncells: tuple
    lo: tuple
    hi: tuple
    p: int
    tree_depth: int
    void_center: np.ndarray
    void_radius: np.ndarray
    alpha: float = 1e-12
    rho: float = 1.0
    c: float = 1.0
    E: float = 1.0
    nu: float = 0.3
    eps: float = 1e-4
    f_lambda: float = 1e-4
    # optional rotated cube (Sec. 3.1): (centre [d], half edge, T [d][d]); the physical
    # domain is then the cube minus the voids
    cube: object = None
    h: float = field(init=False)

    def __post_init__(self):
        self.ncells = tuple(int(n) for n in self.ncells)
        self.lo = tuple(float(x) for x in self.lo)
        self.hi = tuple(float(x) for x in self.hi)
        hs = [(self.hi[k] - self.lo[k]) / self.ncells[k] for k in range(self.dim)]
        if max(hs) - min(hs) > 1e-14 * max(hs):
            raise ValueError("cells must be cubes")
        self.h = hs[0]
        self.void_center = np.asarray(self.void_center, dtype=np.float64).reshape(-1, self.dim)
        self.void_radius = np.asarray(self.void_radius, dtype=np.float64).reshape(-1)
        if self.cube is not None:
            c, a, T = self.cube
            self.cube = (np.asarray(c, dtype=np.float64).reshape(self.dim), float(a),
                         np.asarray(T, dtype=np.float64).reshape(self.dim, self.dim))

    @property
    def nodes_per_dim(self):
        return tuple(n * self.p + 1 for n in self.ncells)

    @property
    def nnodes(self):
        return int(np.prod(self.nodes_per_dim))

    @property
    def ndof(self):
        return self.ncomp * self.nnodes

    @property
    def n_s(self):
        return (self.p + 1) ** self.dim

    @property
    def n_loc(self):
        return self.ncomp * self.n_s

    @staticmethod
    def from_config(cfg):
        keys = ("dim", "ncomp", "ncells", "lo", "hi", "p", "tree_depth", "void_center",
                "void_radius", "alpha", "rho", "c", "E", "nu", "eps", "f_lambda")
        cube = cfg.get("cube")
        if cube is not None:
            cube = (cube["center"], cube["half"], cube["rot"])
        return Problem(**{k: cfg[k] for k in keys}, cube=cube)

    def cell_lo(self, cell):
        """Lower corner of a cell given by its lexicographic index."""
        idx = np.unravel_index(cell, self.ncells[::-1])[::-1]
        return np.array([self.lo[k] + idx[k] * self.h for k in range(self.dim)])

    def cell_node_table(self):
        """(ncells, n_s) global node of each local node of each cell."""
        nd = self.nodes_per_dim
        mi = element.local_multi_index(self.p, self.dim)
        grids = np.meshgrid(*[np.arange(n) for n in self.ncells[::-1]], indexing="ij")
        cidx = [g.ravel() for g in grids[::-1]]
        table = np.zeros((cidx[0].size, mi.shape[0]), dtype=np.int64)
        stride = 1
        for k in range(self.dim):
            table += (cidx[k][:, None] * self.p + mi[None, :, k]) * stride
            stride *= nd[k]
        return table


@dataclass
class Discrete:
    """Everything the explicit step needs, in float64."""
    prob: Problem
    cls: np.ndarray            # per cell: geometry.OUT / UNCUT / CUT (after reclassification)
    cell_nodes: np.ndarray     # (ncells, n_s)
    K_ref: np.ndarray          # (n_loc, n_loc) uncut stiffness
    M_full: np.ndarray         # (n_s, n_s) consistent scalar mass of an uncut cell
    lumped_ref: np.ndarray     # (n_s,) GLL diagonal of an uncut cell
    cut_cells: np.ndarray      # indices of CUT cells
    K_cut: np.ndarray          # (n_cut, n_loc, n_loc)
    Mo_cut: np.ndarray         # (n_cut, n_s, n_s) scalar mass block of each cut cell
    lumped_cut: np.ndarray     # (n_cut, n_s)
    evs_margin: np.ndarray     # (n_cut,)
    evs_nsmall: np.ndarray     # (n_cut,)
    mass: np.ndarray           # (nnodes,) assembled lumped mass per node
    inv_mass: np.ndarray       # (nnodes,) 1/mass on active nodes, 0 elsewhere

    @property
    def uncut_cells(self):
        return np.flatnonzero(self.cls == geometry.UNCUT)

    def cell_dofs(self, cells):
        """(len(cells), n_loc) global DOFs, component-major local order."""
        nodes = self.cell_nodes[cells]
        nn = self.prob.nnodes
        return np.concatenate([nodes + c * nn for c in range(self.prob.ncomp)], axis=1)

    def inv_mass_dof(self):
        return np.tile(self.inv_mass, self.prob.ncomp)


def reference_element(prob):
    """Uncut reference stiffness (GL (p+1)^d, exact), consistent scalar mass M^f and
    the GLL lumped diagonal of a cell (Sec. 2.2)."""
    lo = np.zeros(prob.dim)
    hi = np.full(prob.dim, prob.h)
    pts, wts = element.box_rule(prob.p, lo, hi)
    ones = np.ones(len(wts))
    K, _ = element.element_integrals(prob, lo, pts, wts, ones)
    _, Mf = element.scalar_integrals(prob.p, prob.dim, lo, prob.h, pts, wts, ones,
                                     prob.rho, prob.c)
    return K, Mf, element.gll_lumped_mass(prob.p, prob.dim, prob.h, prob.rho)


def cut_cell_matrices(prob, cell):
    """K_e, scalar M^o_e and the all-void flag of one cut cell (tree quadrature)."""
    lo = prob.cell_lo(cell)
    pts, wts, av, all_void = quadrature.tree_rule(prob.p, lo, lo + prob.h, prob.void_center,
                                                  prob.void_radius, prob.alpha,
                                                  prob.tree_depth, prob.cube)
    K, _ = element.element_integrals(prob, lo, pts, wts, av)
    _, Mo = element.scalar_integrals(prob.p, prob.dim, lo, prob.h, pts, wts, av,
                                     prob.rho, prob.c)
    return K, Mo, all_void


def build(prob, cut_subset=None):
    """Assemble the discrete problem.  ``cut_subset`` limits the (slow) cut-cell
    integration to the given cells - the mass then is not assembled (for sampled
    per-cell checks at full size)."""
    cls = geometry.classify_cells(prob).copy()
    K_ref, Mf, lref = reference_element(prob)
    cand = np.flatnonzero(cls == geometry.CUT)
    if cut_subset is not None:
        cand = np.asarray(cut_subset, dtype=np.int64)
    Ks, Mos, keep = [], [], []
    for cell in cand:
        K, Mo, all_void = cut_cell_matrices(prob, int(cell))
        if all_void:
            cls[cell] = geometry.OUT
            continue
        Ks.append(K)
        Mos.append(Mo)
        keep.append(cell)
    ns, nl = prob.n_s, prob.n_loc
    K_cut = np.array(Ks).reshape(-1, nl, nl)
    Mo_cut = np.array(Mos).reshape(-1, ns, ns)
    lumped, margins, nsmall = [], [], []
    for Mo in Mo_cut:
        d, m, k = stabilize.stabilized_lumped_diagonal(Mo, Mf, prob.eps, prob.f_lambda)
        lumped.append(d)
        margins.append(m)
        nsmall.append(k)
    lumped_cut = np.array(lumped).reshape(-1, ns)
    table = prob.cell_node_table()
    mass = np.zeros(prob.nnodes)
    inv = np.zeros(prob.nnodes)
    if cut_subset is None:
        unc = np.flatnonzero(cls == geometry.UNCUT)
        np.add.at(mass, table[unc], np.broadcast_to(lref, (len(unc), ns)))
        if len(keep):
            np.add.at(mass, table[np.array(keep)], lumped_cut)
        act = mass > 0
        inv[act] = 1.0 / mass[act]
    return Discrete(prob=prob, cls=cls, cell_nodes=table, K_ref=K_ref, M_full=Mf,
                    lumped_ref=lref, cut_cells=np.array(keep, dtype=np.int64),
                    K_cut=K_cut, Mo_cut=Mo_cut, lumped_cut=lumped_cut,
                    evs_margin=np.array(margins), evs_nsmall=np.array(nsmall, dtype=np.int64),
                    mass=mass, inv_mass=inv)


def source_cell_and_values(prob, x):
    """Cell with lo_k <= x_k < lo_k + h in every direction (clamped to the grid) and the
    shape-function values of that cell at x."""
    x = np.asarray(x, dtype=np.float64)
    idx = []
    for k in range(prob.dim):
        i = int(math.floor((x[k] - prob.lo[k]) / prob.h))
        idx.append(min(max(i, 0), prob.ncells[k] - 1))
    cell = 0
    stride = 1
    for k in range(prob.dim):
        cell += idx[k] * stride
        stride *= prob.ncells[k]
    lo = prob.cell_lo(cell)
    N, _ = element.physical_shape(prob.p, prob.dim, lo, prob.h, x[None, :])
    return cell, N[0]


def gaussian_support(prob, cls, x, sigma):
    """Active cells (not OUT) whose box comes closer than 8 sigma to x (squared distance
    from x to the box below 64 sigma^2), in increasing cell order."""
    x = np.asarray(x, dtype=np.float64)
    cells = []
    for cell in np.flatnonzero(cls != geometry.OUT):
        lo = prob.cell_lo(int(cell))
        d2 = 0.0
        for k in range(prob.dim):
            gap = max(lo[k] - x[k], 0.0, x[k] - (lo[k] + prob.h))
            d2 = d2 + gap * gap
        if d2 < 64.0 * sigma * sigma:
            cells.append(int(cell))
    return np.array(cells, dtype=np.int64)


def gaussian_load(disc, src):
    """Spatial part b of a volumetric Gaussian source (Sec. 3.1; dict with x, sigma, amp,
    dir): f(x, t) = f_t(t) amp exp(-|x - x_s|^2 / (2 sigma^2)), so by eq.
    weak_form_extended b_i = int alpha^FCM rho amp exp(...) N_i dx (times dir_c for
    elasticity).  Reading of the quadrature (the paper does not state it): the active
    cells within 8 sigma of x_s (``gaussian_support``; the Gaussian is below e^-32 beyond),
    each split into m^d equal boxes with m = ceil(h / sigma) (at most 64), a Gauss-Legendre rule of
    p + 3 points per direction on every box, the indicator alpha^FCM at every point."""
    prob = disc.prob
    xs = np.asarray(src["x"], dtype=np.float64)
    sigma = float(src["sigma"])
    amp = float(src.get("amp", 1.0))
    direction = np.asarray(src.get("dir", (1.0,)), dtype=np.float64)
    m = max(1, min(64, int(math.ceil(prob.h / sigma))))
    xq, wq = basis.gl_points(prob.p + 3)
    b = np.zeros(prob.ndof)
    for cell in gaussian_support(prob, disc.cls, xs, sigma):
        lo = prob.cell_lo(int(cell))
        sub = prob.h / m
        pts, wts = [], []
        for idx in np.ndindex(*(m,) * prob.dim):
            blo = lo + sub * np.array(idx[::-1], dtype=np.float64)
            grids = [blo[k] + 0.5 * sub * (xq + 1.0) for k in range(prob.dim)]
            mesh = np.meshgrid(*grids[::-1], indexing="ij")
            pts.append(np.stack([g.ravel() for g in mesh[::-1]], axis=1))
            wmesh = np.meshgrid(*([wq * (0.5 * sub)] * prob.dim), indexing="ij")
            w = np.ones(wmesh[0].size)
            for g in wmesh:
                w = w * g.ravel()
            wts.append(w)
        pts = np.concatenate(pts)
        wts = np.concatenate(wts)
        r2 = np.zeros(len(wts))
        for k in range(prob.dim):
            r2 = r2 + (pts[:, k] - xs[k]) ** 2
        g = np.exp(-0.5 * r2 / (sigma * sigma))
        al = geometry.indicator(pts, prob.void_center, prob.void_radius, prob.alpha, prob.cube)
        N, _ = element.physical_shape(prob.p, prob.dim, lo, prob.h, pts)
        be = prob.rho * amp * ((wts * al * g) @ N)
        for comp in range(prob.ncomp):
            dcomp = direction[comp] if prob.ncomp > 1 else 1.0
            np.add.at(b, disc.cell_nodes[cell] + comp * prob.nnodes, dcomp * be)
    return b


def load_vector(disc, src):
    """Spatial part b of F(t) = f_t(t) b for one source: a point source (dict with x, dir,
    amp), or a volumetric Gaussian when the dict has sigma > 0 (``gaussian_load``)."""
    if float(src.get("sigma", 0.0)) > 0.0:
        return gaussian_load(disc, src)
    prob = disc.prob
    cell, N = source_cell_and_values(prob, src["x"])
    b = np.zeros(prob.ndof)
    direction = np.asarray(src.get("dir", (1.0,)), dtype=np.float64)
    for comp in range(prob.ncomp):
        dcomp = direction[comp] if prob.ncomp > 1 else 1.0
        np.add.at(b, disc.cell_nodes[cell] + comp * prob.nnodes,
                  prob.rho * src.get("amp", 1.0) * dcomp * N)
    return b


def receiver_rows(disc, points):
    """Observers (Sec. 3.2, observer traces): a matrix R with one row per (point, component),
    row r * ncomp + comp, such that (R u)[row] = u_h(x_r) of that component, the finite
    element field sum_a N_a(x_r) u_a of a cell containing x_r (the cell rule of the point
    sources; the field is continuous, so any such cell gives the same row)."""
    prob = disc.prob
    pts = np.asarray(points, dtype=np.float64).reshape(-1, prob.dim)
    R = np.zeros((len(pts) * prob.ncomp, prob.ndof))
    for r, x in enumerate(pts):
        cell, N = source_cell_and_values(prob, x)
        for comp in range(prob.ncomp):
            R[r * prob.ncomp + comp, disc.cell_nodes[cell] + comp * prob.nnodes] = N
    return R


def ricker(t, f0):
    """Ricker wavelet, eq. source_time: (1 - 2 q^2) exp(-q^2), q = pi f0 (t - t_s),
    t_s = 2 sqrt(6) / (pi f0)."""
    ts = 2.0 * math.sqrt(6.0) / (math.pi * f0)
    q = math.pi * f0 * (t - ts)
    return (1.0 - 2.0 * q * q) * math.exp(-q * q)


def _cell_dof_tables(disc):
    """(uncut DOF table, cut DOF table) as torch int64 tensors, built once per problem."""
    import torch
    cached = getattr(disc, "_dof_tables", None)
    if cached is None:
        cached = tuple(torch.from_numpy(np.ascontiguousarray(disc.cell_dofs(cells)))
                       for cells in (disc.uncut_cells, disc.cut_cells))
        disc._dof_tables = cached
    return cached


def apply_K(disc, u, out=None):
    """K u element by element (eq. semi): the sum over uncut cells of P_e^T K_ref P_e u
    plus the cut cells with their own matrices.  The gather P_e u, the element products
    and the scatter-add P_e^T are torch CPU indexing, matmul and index_add (library
    primitives; the order in which the element contributions add up at a node is left to
    the library).  u: (ndof,) or (ndof, nrhs); ``out`` (same shape) receives the result."""
    import torch
    u = np.asarray(u, dtype=np.float64)
    vec = u.ndim == 1
    U = torch.from_numpy(np.ascontiguousarray(u[:, None] if vec else u))
    if out is None:
        res = np.zeros(u.shape)
    else:
        res = out
        res[...] = 0.0
    R = torch.from_numpy(res[:, None] if vec else res)
    for dofs, mats in zip(_cell_dof_tables(disc), (None, disc.K_cut)):
        if dofs.shape[0] == 0:
            continue
        ue = U[dofs]                                        # (cells, n_loc, nrhs)
        if mats is None:
            ye = torch.matmul(torch.from_numpy(disc.K_ref), ue)
        else:
            ye = torch.bmm(torch.from_numpy(mats), ue)
        R.index_add_(0, dofs.reshape(-1), ye.reshape(-1, U.shape[1]))
    return res


def assembled_K(disc):
    """Global sparse stiffness (for eigenvalue checks)."""
    prob = disc.prob
    rows, cols, vals = [], [], []
    for cells, mats in ((disc.uncut_cells, None), (disc.cut_cells, disc.K_cut)):
        if len(cells) == 0:
            continue
        dofs = disc.cell_dofs(cells)
        for e in range(len(cells)):
            Ke = disc.K_ref if mats is None else mats[e]
            rows.append(np.repeat(dofs[e], len(dofs[e])))
            cols.append(np.tile(dofs[e], len(dofs[e])))
            vals.append(Ke.ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(prob.ndof, prob.ndof))
    return K.tocsr()
