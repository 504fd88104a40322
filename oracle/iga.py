"""IGA-FCM: the immersed problem discretised with B-splines (paper Sec. 2.2: B-spline shape
functions give the isogeometric variant of the finite cell method; Sec. 2.4: row-sum
lumping; Table methods: IGA-FCM with alpha stabilisation and epsilon = 0, central
differences).

Readings (the paper names the basis but does not spell the spline space out):
  * degree p, maximum continuity C^{p-1}, one open uniform knot vector per direction:
    p + 1 copies of each end of the box and the n - 1 interior cell faces, so n cells
    along a direction carry n + p basis functions and cell c (the knot span [t_{c+p},
    t_{c+p+1}]) supports the functions c .. c + p;
  * tensor products in 2-D and 3-D, DOF = i0 + n0' (i1 + n1' i2) with n_k' = n_k + p and
    the local functions of a cell ordered x fastest (as the SCM cell's nodes);
  * integration as in the SCM: the Gauss-Legendre (p+1)^d rule in uncut cells (the
    restrictions of the B-splines to a cell are polynomials of degree p per direction, so
    the rule is exact for stiffness and mass), the space tree of ``quadrature`` in cut
    cells; a cut cell whose tree finds only void is dropped like a cell outside;
  * row-sum lumping (Sec. 2.4): m_i = sum_j M_ij = int alpha rho N_i.  B-splines form a
    nonnegative partition of unity, so every lumped mass is >= 0 and an active DOF (one
    supported by a kept cell, alpha > 0) has a positive mass; inactive DOFs stay zero;
  * the point load b_i = rho amp N_i(x_s) is taken in the cell containing x_s (the rule
    of the SCM's point sources; the basis is continuous, so any such cell gives the same
    vector).

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import element, geometry, quadrature
from .problem import ricker
from .timestep import _cdm_loop


def knot_vector(n, p, lo, h):
    """Open uniform knot vector of n cells of width h starting at lo (p + 1 end copies)."""
    inner = [lo + k * h for k in range(1, n)]
    hi = lo + n * h
    return np.array([lo] * (p + 1) + inner + [hi] * (p + 1), dtype=np.float64)


def _span(t, p, nb, x):
    """Knot span index s (t_s <= x < t_{s+1}, p <= s <= nb - 1) of each point; the right
    end of the knot vector belongs to the last span."""
    s = np.searchsorted(t, x, side="right") - 1
    return np.clip(s, p, nb - 1)


def bspline_values(t, p, x, span=None):
    """Values of all basis functions of degree p on knot vector t at points x, by the
    Cox-de Boor recursion from the degree-0 indicators of the knot spans (0/0 := 0).
    ``span`` (optional) forces the knot span whose polynomial pieces are evaluated (a
    point on a span's end then takes that span's pieces).  Returns (len(x), len(t)-p-1)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nb = len(t) - p - 1
    s = _span(t, p, nb, x) if span is None else np.full(len(x), int(span))
    N = np.zeros((len(x), len(t) - 1))
    N[np.arange(len(x)), s] = 1.0
    for q in range(1, p + 1):
        new = np.zeros((len(x), len(t) - 1 - q))
        for i in range(len(t) - 1 - q):
            d1 = t[i + q] - t[i]
            d2 = t[i + q + 1] - t[i + 1]
            if d1 > 0.0:
                new[:, i] += (x - t[i]) / d1 * N[:, i]
            if d2 > 0.0:
                new[:, i] += (t[i + q + 1] - x) / d2 * N[:, i + 1]
        N = new
    return N


def bspline_derivatives(t, p, x, span=None):
    """First derivatives of the degree-p basis functions at x:
    N'_{i,p} = p N_{i,p-1} / (t_{i+p} - t_i) - p N_{i+1,p-1} / (t_{i+p+1} - t_{i+1})."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nb = len(t) - p - 1
    if p == 0:
        return np.zeros((len(x), nb))
    low = bspline_values(t, p - 1, x, span)  # (len(x), nb + 1)
    out = np.zeros((len(x), nb))
    for i in range(nb):
        d1 = t[i + p] - t[i]
        d2 = t[i + p + 1] - t[i + 1]
        if d1 > 0.0:
            out[:, i] += p * low[:, i] / d1
        if d2 > 0.0:
            out[:, i] -= p * low[:, i + 1] / d2
    return out


@dataclass
class IgaDiscrete:
    """Everything the explicit IGA-FCM step needs, in float64."""
    prob: object
    cls: np.ndarray          # per cell: OUT / UNCUT / CUT (after dropping all-void cut cells)
    nbasis: tuple            # basis functions per direction (n_k + p)
    cell_dofs: np.ndarray    # (ncells, n_s) global DOF of each local function
    cells: np.ndarray        # kept (UNCUT or CUT) cells, ascending
    K_cells: np.ndarray      # (len(cells), n_s, n_s) element stiffness
    M_cells: np.ndarray      # (len(cells), n_s, n_s) element consistent mass
    mass: np.ndarray         # (ndof,) row-sum lumped mass
    inv_mass: np.ndarray     # (ndof,) 1 / mass on active DOFs, 0 elsewhere

    @property
    def ndof(self):
        return int(np.prod(self.nbasis))


def knots(prob):
    """The knot vector of each direction."""
    return [knot_vector(prob.ncells[k], prob.p, prob.lo[k], prob.h) for k in range(prob.dim)]


def cell_dof_table(prob):
    """(ncells, n_s) global DOFs of every cell's local functions (x fastest)."""
    nb = [n + prob.p for n in prob.ncells]
    mi = element.local_multi_index(prob.p, prob.dim)
    grids = np.meshgrid(*[np.arange(n) for n in prob.ncells[::-1]], indexing="ij")
    cidx = [g.ravel() for g in grids[::-1]]
    table = np.zeros((cidx[0].size, mi.shape[0]), dtype=np.int64)
    stride = 1
    for k in range(prob.dim):
        table += (cidx[k][:, None] + mi[None, :, k]) * stride
        stride *= nb[k]
    return table


def cell_index(prob, cell):
    """Cell coordinates (c0, c1[, c2]) of a lexicographic cell index."""
    return np.unravel_index(cell, prob.ncells[::-1])[::-1]


def cell_shape(prob, kv, cell, pts):
    """Values N (npts, n_s) and gradients G (npts, dim, n_s) of the p + 1 (per direction)
    B-splines supported on ``cell`` at physical points inside it: tensor products of the
    1-D functions c_k .. c_k + p of each direction."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    ci = cell_index(prob, cell)
    p, dim = prob.p, prob.dim
    mi = element.local_multi_index(p, dim)
    vals, ders = [], []
    for k in range(dim):
        # functions c .. c + p depend on the knots t_c .. t_{c+2p+1} only: the recursion
        # runs on that slice, where the cell's own knot span (span c + p of the whole
        # vector, also for a point on the cell's upper face) is span p
        c = int(ci[k])
        x = pts[:, k]
        t = kv[k][c:c + 2 * p + 2]
        vals.append(bspline_values(t, p, x, span=p))
        ders.append(bspline_derivatives(t, p, x, span=p))
    npts, ns = pts.shape[0], mi.shape[0]
    N = np.ones((npts, ns))
    G = np.ones((npts, dim, ns))
    for a in range(dim):
        N *= vals[a][:, mi[:, a]]
        for b in range(dim):
            G[:, b, :] *= (ders[a] if a == b else vals[a])[:, mi[:, a]]
    return N, G


def element_matrices(prob, kv, cell, pts, wts, alpha_vals):
    """K_ij = sum_q w_q a_q rho c^2 grad N_i . grad N_j and M_ij = sum_q w_q a_q rho N_i N_j
    (eq. weak_form_extended with the B-spline basis)."""
    N, G = cell_shape(prob, kv, cell, pts)
    wa = np.asarray(wts) * np.asarray(alpha_vals)
    K = prob.rho * prob.c * prob.c * np.tensordot(G * wa[:, None, None], G, axes=([0, 1], [0, 1]))
    M = prob.rho * np.einsum("q,qi,qj->ij", wa, N, N)
    return K, M


def cell_matrices(prob, kv, cell, cls_value):
    """(K, M) of one cell of class cls_value (UNCUT: the GL rule; CUT: the space tree), or
    None for a cut cell whose tree finds only void (the cell is then dropped)."""
    lo = prob.cell_lo(int(cell))
    hi = lo + prob.h
    if cls_value == geometry.UNCUT:
        pts, wts = element.box_rule(prob.p, lo, hi)
        av = np.ones(len(wts))
    else:
        pts, wts, av, all_void = quadrature.tree_rule(prob.p, lo, hi, prob.void_center,
                                                      prob.void_radius, prob.alpha,
                                                      prob.tree_depth, prob.cube)
        if all_void:
            return None
    return element_matrices(prob, kv, int(cell), pts, wts, av)


def build(prob):
    """Assemble the IGA-FCM problem of a scalar ``Problem`` (its p, grid, voids, cube,
    alpha, rho, c, tree depth)."""
    if prob.ncomp != 1:
        raise ValueError("IGA-FCM is built for the scalar wave equation")
    cls = geometry.classify_cells(prob).copy()
    kv = knots(prob)
    Ks, Ms, keep = [], [], []
    for cell in np.flatnonzero(cls != geometry.OUT):
        km = cell_matrices(prob, kv, int(cell), cls[cell])
        if km is None:
            cls[cell] = geometry.OUT
            continue
        K, M = km
        Ks.append(K)
        Ms.append(M)
        keep.append(int(cell))
    ns = (prob.p + 1) ** prob.dim
    nb = tuple(n + prob.p for n in prob.ncells)
    table = cell_dof_table(prob)
    cells = np.array(keep, dtype=np.int64)
    K_cells = np.array(Ks).reshape(-1, ns, ns)
    M_cells = np.array(Ms).reshape(-1, ns, ns)
    mass = np.zeros(int(np.prod(nb)))
    if len(cells):
        np.add.at(mass, table[cells], M_cells.sum(axis=2))
    inv = np.zeros_like(mass)
    act = mass > 0
    inv[act] = 1.0 / mass[act]
    return IgaDiscrete(prob=prob, cls=cls, nbasis=nb, cell_dofs=table, cells=cells,
                       K_cells=K_cells, M_cells=M_cells, mass=mass, inv_mass=inv)


def apply_K(disc, u, out=None):
    """K u as the sum over kept cells of P_e^T K_e P_e u (eq. semi); u: (ndof,) or
    (ndof, nrhs).  The gather, the element products and the scatter-add are numpy
    indexing, matmul and add.at."""
    u = np.asarray(u, dtype=np.float64)
    res = np.zeros(u.shape) if out is None else out
    res[...] = 0.0
    if len(disc.cells) == 0:
        return res
    dofs = disc.cell_dofs[disc.cells]
    ue = u[dofs]                                  # (cells, n_s[, nrhs])
    ye = np.matmul(disc.K_cells, ue if u.ndim > 1 else ue[..., None])
    if u.ndim == 1:
        ye = ye[..., 0]
    np.add.at(res, dofs, ye)
    return res


def assembled(disc):
    """Dense assembled K and consistent M (small problems; for eigenvalue and stencil
    checks)."""
    n = disc.ndof
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    for e, cell in enumerate(disc.cells):
        d = disc.cell_dofs[cell]
        K[np.ix_(d, d)] += disc.K_cells[e]
        M[np.ix_(d, d)] += disc.M_cells[e]
    return K, M


def source_values(prob, x):
    """Cell containing x (lo_k <= x_k < lo_k + h, clamped to the grid) and the values of
    its B-splines at x."""
    x = np.asarray(x, dtype=np.float64)
    cell, stride = 0, 1
    for k in range(prob.dim):
        i = int(math.floor((x[k] - prob.lo[k]) / prob.h))
        cell += min(max(i, 0), prob.ncells[k] - 1) * stride
        stride *= prob.ncells[k]
    N, _ = cell_shape(prob, knots(prob), cell, x[None, :])
    return cell, N[0]


def load_vector(disc, src):
    """b_i = rho amp N_i(x_s) of a point source (dict with x, amp)."""
    cell, N = source_values(disc.prob, src["x"])
    b = np.zeros(disc.ndof)
    np.add.at(b, disc.cell_dofs[cell], disc.prob.rho * src.get("amp", 1.0) * N)
    return b


def critical_dt(disc):
    """dt_crit = 2 / sqrt(lambda_max) of the lumped system (Sec. 2.3), lambda_max the
    largest eigenvalue of M^{-1/2} K M^{-1/2} over the active DOFs (dense eigvalsh)."""
    K, _ = assembled(disc)
    act = np.flatnonzero(disc.inv_mass > 0)
    s = np.sqrt(disc.inv_mass[act])
    A = K[np.ix_(act, act)] * s[:, None] * s[None, :]
    lam = float(np.linalg.eigvalsh(0.5 * (A + A.T))[-1])
    return 2.0 / math.sqrt(lam)


def cdm(disc, dt, nsteps, sources=(), u0=None, v0=None, t0=0.0):
    """Central differences (eq. cdm) with the row-sum lumped mass and the Newmark
    (beta = 0) start-up, in the form of ``timestep.cdm``.  Returns dict(u, u_prev, k)."""
    n = disc.ndof
    im = disc.inv_mass
    u = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros(n) if v0 is None else np.array(v0, dtype=np.float64)
    loads = []
    for s in sources:
        b = load_vector(disc, s)
        nz = np.flatnonzero(b)
        loads.append((nz, b[nz], float(s.get("f0", 10.0))))

    def accel(k, u_k, out):
        apply_K(disc, u_k, out=out)
        np.negative(out, out=out)
        for nz, bv, f0 in loads:
            out[nz] += ricker(t0 + k * dt, f0) * bv
        out *= im
        return out

    if nsteps == 0:
        return dict(u=u, u_prev=u - dt * v, k=0)
    a = accel(0, u, np.empty(n))
    u_prev = u
    u = u + dt * v + 0.5 * dt * dt * a
    res = _cdm_loop(1, nsteps, u_prev.copy(), u, a, accel, dt, (), {}, None, [], None)
    return dict(u=res["u"], u_prev=res["u_prev"], k=res["k"])


def energy(disc, u_k, u_k1, dt):
    """Discrete energy 1/2 v^T M v + 1/2 u_{k+1}^T K u_k with the lumped mass (conserved
    by eq. cdm without load, as for the SCM)."""
    v = (u_k1 - u_k) / dt
    return 0.5 * float(v @ (disc.mass * v)) + 0.5 * float(u_k1 @ apply_K(disc, u_k))
