"""Eigenvalue (epsilon) stabilisation and HRZ lumping of cut-cell mass matrices
(paper Sec. 2.6, eqs. epsilon_stabilization / alpha_stabilization and the M^s
construction; Sec. 2.4, HRZ lumping).

Readings where the paper is silent:
  * The decomposed matrix is the original cut-cell mass M^o *including* the alpha
    part of the indicator (the paper reports the eigensolver failing without alpha).
  * max(A) is the largest entry of A; M^f is the consistent mass of an uncut cell
    integrated with the same rule as M^o.
  * The explicit path needs a diagonal mass.  The stabilised lumped diagonal of a cut
    cell is HRZ(M^o) + eps * diag(M^s), where HRZ uses m^e = sum_ij M^o_ij (the
    alpha-weighted element mass, by partition of unity).
  * Vector problems decompose the scalar mass block; the vector mass is that block
    repeated on every component, so its lumped diagonal is the scalar one repeated.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np


def evs_matrix(Mo, Mf, f_lambda):
    """Stabilisation matrix M^s of Sec. 2.6 and the classification margin.

    M^o = Phi Lambda Phi^T (eigh); small set S = {i : lambda_i < f_lambda lambda_max};
    M~^s = Phi_S Phi_S^T;  M^s = max(M^f)/max(M~^s) M~^s  (0 if S is empty).
    The margin min_i |lambda_i/lambda_max - f_lambda| tells how far the split is from
    being decided by rounding.
    """
    lam, phi = np.linalg.eigh(Mo)
    lmax = lam[-1]
    small = lam < f_lambda * lmax
    margin = float(np.min(np.abs(lam / lmax - f_lambda)))
    if not np.any(small):
        return np.zeros_like(Mo), margin, 0
    ps = phi[:, small]
    mt = ps @ ps.T
    ms = (np.max(Mf) / np.max(mt)) * mt
    return ms, margin, int(np.count_nonzero(small))


def hrz_diagonal(M, total_mass):
    """HRZ (diagonal scaling) lumping, Sec. 2.4:  m~_ii = m^e / sum_j m_jj * m_ii."""
    d = np.diag(M).copy()
    return total_mass / np.sum(d) * d


def stabilized_lumped_diagonal(Mo_scalar, Mf_scalar, eps, f_lambda):
    """Lumped diagonal of one cut cell: HRZ(M^o) + eps diag(M^s) (scalar block).

    Returns (diag, margin, n_small).
    """
    ms, margin, nsmall = evs_matrix(Mo_scalar, Mf_scalar, f_lambda)
    d = hrz_diagonal(Mo_scalar, float(np.sum(Mo_scalar))) + eps * np.diag(ms)
    return d, margin, nsmall
