"""Newmark IMEX time integration (paper Sec. 2.5, Alg. imex).

The DOFs split by the support of their basis functions: a DOF whose node lies only in
uncut cells is explicit ("d"); a DOF whose node lies in at least one cut cell is
implicit ("c").  With GLL nodes and nodal quadrature the mass of an uncut cell is
diagonal, so M = diag(M^dd, M^cc) with M^dd diagonal and M^cc the consistent mass of the
cut DOFs: the original tree-integrated cut-cell masses M^o_e (no stabilisation) plus
the GLL diagonals of the uncut cells that touch cut DOFs.  The explicit DOFs take the
central difference step, the implicit ones the trapezoidal Newmark step (beta = 1/4,
gamma = 1/2) with S = M^cc + beta dt^2 K^cc, whose right-hand side uses the explicit
DOFs' new values as their predictors.

Readings (where the algorithm as printed is silent):
* the explicit part's first step uses the Newmark start-up with beta = 0 (as the
  explicit solver does), since Alg. imex needs Psi_{-1};
* the initial acceleration of the implicit DOFs solves M^cc a_0 = F_0^c - K^c Psi_0
  (the printed line writes F_k for F_0);
* F_{k+1} in the implicit step is the load at t_{k+1}.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .problem import assembled_K, load_vector, ricker


def partition(disc):
    """(c, d): sorted global DOF indices of the implicit DOFs (nodes of cut cells, every
    component) and of the remaining active DOFs."""
    prob = disc.prob
    nn = prob.nnodes
    cut_nodes = np.zeros(nn, dtype=bool)
    if len(disc.cut_cells):
        cut_nodes[disc.cell_nodes[disc.cut_cells].ravel()] = True
    active = disc.mass > 0
    c_nodes = np.flatnonzero(cut_nodes & active)
    d_nodes = np.flatnonzero(active & ~cut_nodes)
    c = np.concatenate([c_nodes + k * nn for k in range(prob.ncomp)])
    d = np.concatenate([d_nodes + k * nn for k in range(prob.ncomp)])
    return c, d


def mass_matrices(disc, c, d):
    """(m_dd, M_cc): the diagonal of M^dd (GLL diagonals of the uncut cells) and the
    consistent M^cc (cut-cell M^o_e blocks, one per component, plus the uncut-cell GLL
    diagonals on cut DOFs), both in the order of c and d."""
    prob = disc.prob
    nn, ns = prob.nnodes, prob.n_s
    diag = np.zeros(nn)
    unc = disc.uncut_cells
    if len(unc):
        np.add.at(diag, disc.cell_nodes[unc], np.broadcast_to(disc.lumped_ref, (len(unc), ns)))
    rows, cols, vals = [], [], []
    for e, cell in enumerate(disc.cut_cells):
        nodes = disc.cell_nodes[cell]
        for k in range(prob.ncomp):
            g = nodes + k * nn
            rows.append(np.repeat(g, ns))
            cols.append(np.tile(g, ns))
            vals.append(disc.Mo_cut[e].ravel())
    full_diag = np.tile(diag, prob.ncomp)
    ndof = prob.ndof
    M = sp.coo_matrix((np.concatenate(vals + [full_diag]),
                       (np.concatenate(rows + [np.arange(ndof)]),
                        np.concatenate(cols + [np.arange(ndof)]))), shape=(ndof, ndof)).tocsr()
    return full_diag[d], M[c][:, c]


def imex(disc, dt, nsteps, sources=(), beta=0.25, gamma=0.5, t0=0.0, split=None, u0=None,
         sparse=False):
    """Run ``nsteps`` steps of the IMEX scheme of Sec. 2.5 from u0 (default 0) at rest.
    ``split`` overrides the partition (c, d) (a test reduces the scheme to one of its two
    parts with it).  Returns the final u (all DOFs), the implicit DOFs' velocity and
    acceleration, and the split.  The solves with S and M^cc use a dense Cholesky factor,
    or with ``sparse`` a sparse LU factor (SuperLU) of the same matrices, for implicit
    sets too large for a dense one.

    The explicit DOFs take eq. cdm.  The implicit DOFs take the Newmark relations
        u_{k+1} = u_k + dt v_k + dt^2 ((1/2 - beta) a_k + beta a_{k+1}),
        v_{k+1} = v_k + dt ((1 - gamma) a_k + gamma a_{k+1}),
        M^cc a_{k+1} = F^c_{k+1} - K^cc u^c_{k+1} - K^cd u^d_{k+1},
    with u^d_{k+1} the explicit DOFs' new values.  Eliminating a_{k+1} with the first
    relation gives the implicit displacements from one solve with S = M^cc + beta dt^2 K^cc:
        S u^c_{k+1} = M^cc w + beta dt^2 (F^c_{k+1} - K^cd u^d_{k+1}),
        w = u^c_k + dt v_k + (1/2 - beta) dt^2 a_k,
    after which a_{k+1} = (u^c_{k+1} - w) / (beta dt^2) and the velocity follows."""
    prob = disc.prob
    c, d = partition(disc) if split is None else split
    m_dd, Mcc = mass_matrices(disc, c, d)
    K = assembled_K(disc)
    Kcc = K[c][:, c]
    Kcd = K[c][:, d]
    Kd = K[d]
    loads = [(load_vector(disc, s), float(s.get("f0", 10.0))) for s in sources]

    def force(k):
        F = np.zeros(prob.ndof)
        for b, f0 in loads:
            F += ricker(t0 + k * dt, f0) * b
        return F

    u = np.zeros(prob.ndof) if u0 is None else np.array(u0, dtype=np.float64)
    v_c = np.zeros(len(c))
    a_c = np.zeros(len(c))
    bdt2 = beta * dt * dt
    if len(c) and sparse:
        Mc = (0.5 * (Mcc + Mcc.T)).tocsc()
        S = (Mc + bdt2 * Kcc).tocsc()
        S_lu = spla.splu((0.5 * (S + S.T)).tocsc())
        solve_S = S_lu.solve
        # initial acceleration from the equation of motion at t_0
        a_c = spla.splu(Mc).solve(force(0)[c] - K[c] @ u)
    elif len(c):
        Mc = Mcc.toarray()
        Mc = 0.5 * (Mc + Mc.T)
        S = Mc + bdt2 * Kcc.toarray()
        S_f = sla.cho_factor(0.5 * (S + S.T), lower=True)

        def solve_S(rhs):
            return sla.cho_solve(S_f, rhs)
        # initial acceleration from the equation of motion at t_0
        a_c = sla.cho_solve(sla.cho_factor(Mc, lower=True), force(0)[c] - K[c] @ u)
    inv_dd = np.where(m_dd > 0, 1.0 / np.where(m_dd > 0, m_dd, 1.0), 0.0)
    ud_prev = None
    for k in range(nsteps):
        Fk = force(k)
        # explicit DOFs: eq. cdm, the first step by the Newmark rule with beta = 0
        acc_d = inv_dd * (Fk[d] - Kd @ u)
        if k == 0:
            ud_new = u[d] + 0.5 * dt * dt * acc_d
        else:
            ud_new = 2.0 * u[d] - ud_prev + dt * dt * acc_d
        ud_prev = u[d].copy()
        u_new = u.copy()
        u_new[d] = ud_new
        if len(c):
            w = u[c] + dt * v_c + (0.5 - beta) * dt * dt * a_c
            rhs = Mc @ w + bdt2 * (force(k + 1)[c] - Kcd @ ud_new)
            uc_new = solve_S(rhs)
            a_new = (uc_new - w) / bdt2
            v_c = v_c + dt * ((1.0 - gamma) * a_c + gamma * a_new)
            a_c = a_new
            u_new[c] = uc_new
        u = u_new
    return dict(u=u, v_c=v_c, a_c=a_c, c=c, d=d)


def cdm_consistent(disc, dt, nsteps, sources=(), t0=0.0, u0=None):
    """Central differences (eq. cdm, Newmark beta = 0 start-up) with the block mass
    M = diag(M^dd, M^cc) of the split above: the consistent cut-DOF mass is solved for
    every step, the explicit DOFs keep their diagonal.  Returns the final and the previous
    u."""
    prob = disc.prob
    c, d = partition(disc)
    m_dd, Mcc = mass_matrices(disc, c, d)
    K = assembled_K(disc)
    loads = [(load_vector(disc, s), float(s.get("f0", 10.0))) for s in sources]

    def force(k):
        F = np.zeros(prob.ndof)
        for b, f0 in loads:
            F += ricker(t0 + k * dt, f0) * b
        return F

    Mc_f = None
    if len(c):
        Mc = Mcc.toarray()
        Mc_f = sla.cho_factor(0.5 * (Mc + Mc.T), lower=True)
    inv_dd = np.where(m_dd > 0, 1.0 / np.where(m_dd > 0, m_dd, 1.0), 0.0)

    def accel(k, u):
        r = force(k) - K @ u
        a = np.zeros(prob.ndof)
        a[d] = inv_dd * r[d]
        if len(c):
            a[c] = sla.cho_solve(Mc_f, r[c])
        return a

    u = np.zeros(prob.ndof) if u0 is None else np.array(u0, dtype=np.float64)
    u_prev = u.copy()
    for k in range(nsteps):
        a = accel(k, u)
        if k == 0:
            u_next = u + 0.5 * dt * dt * a
        else:
            u_next = 2.0 * u - u_prev + dt * dt * a
        u_prev, u = u, u_next
    return dict(u=u, u_prev=u_prev, c=c, d=d)
