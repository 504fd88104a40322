"""Time integration of M u'' + K u = F (paper Sec. 2.3).

* Critical step of the central difference method: dt_crit = 2 / sqrt(lambda_max(K, M)).
* Central differences, eq. cdm:  u_{k+1} = 2 u_k - u_{k-1} + dt^2 M^{-1} (F_k - K u_k),
  started as the Newmark predictor-corrector with beta = 0, gamma = 1/2 (Alg. newmark):
  a_0 = M^{-1}(F_0 - K u_0),  u_1 = u_0 + dt v_0 + dt^2/2 a_0.

M is the assembled diagonal (lumped) mass; DOFs without mass are inactive and kept 0.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from .problem import apply_K, assembled_K, load_vector, ricker


def lambda_max(disc, dense_limit=6000, tol=1e-12):
    """Largest eigenvalue of the generalized problem K x = lambda M x over the active
    DOFs, as the largest eigenvalue of M^{-1/2} K M^{-1/2}: dense eigvalsh for small
    problems, ARPACK Lanczos (eigsh) otherwise."""
    prob = disc.prob
    im = disc.inv_mass_dof()
    act = np.flatnonzero(im > 0)
    s = np.sqrt(im[act])
    if len(act) <= dense_limit:
        K = assembled_K(disc)[act][:, act]
        A = (K.toarray() * s[:, None]) * s[None, :]
        return float(np.linalg.eigvalsh(0.5 * (A + A.T))[-1])
    # x -> M^{-1/2} K M^{-1/2} x on the active DOFs, K applied element by element
    full = np.zeros(prob.ndof)
    ku = np.zeros(prob.ndof)

    def matvec(x):
        full[act] = s * np.ravel(x)
        apply_K(disc, full, out=ku)
        return s * ku[act]

    A = spla.LinearOperator((len(act), len(act)), matvec=matvec, dtype=np.float64)
    v0 = np.ones(len(act))
    vals = spla.eigsh(A, k=1, which="LA", tol=tol, v0=v0, return_eigenvectors=False,
                      ncv=64, maxiter=20000)
    return float(vals[-1])


def critical_dt(disc, **kw):
    """dt_crit = 2 / sqrt(lambda_max) (Sec. 2.3)."""
    return 2.0 / math.sqrt(lambda_max(disc, **kw))


def cdm(disc, dt, nsteps, sources=(), u0=None, v0=None, t0=0.0, checkpoints=(),
        receivers=None, progress=None, resume=None):
    """Run ``nsteps`` central-difference steps (eq. cdm) with the Newmark (beta=0)
    start-up.  ``sources``: list of dicts (x, dir, amp, f0); every source adds
    f_t(t_k) b to F_k.  Several right-hand sides are run by calling this once per
    source set.  Returns dict with the final u, the previous u, the states at the
    requested checkpoint step numbers, and receiver traces (one row per step k=0..n).
    ``progress(k)``, if given, is called after step k.  ``resume``: the dict returned by
    an earlier call with the same disc, dt, sources and t0; the run then continues
    from its last step (no start-up) up to step ``nsteps`` of the whole run.

    Each step works in place on three state-sized arrays (a point load is nonzero on
    one cell's DOFs only, so F_k is added where it is nonzero):
        a   = M^{-1} (F_k - K u_k)
        u_{k+1} = 2 u_k - u_{k-1} + dt^2 a   (written over u_{k-1}).
    """
    prob = disc.prob
    im = disc.inv_mass_dof()
    u = np.zeros(prob.ndof) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros(prob.ndof) if v0 is None else np.array(v0, dtype=np.float64)
    loads = []
    for s in sources:
        b = load_vector(disc, s)
        nz = np.flatnonzero(b)
        loads.append((nz, b[nz], float(s.get("f0", 10.0))))

    def accel(k, u_k, out):
        """out = M^{-1} (F_k - K u_k)."""
        apply_K(disc, u_k, out=out)
        np.negative(out, out=out)
        for nz, bv, f0 in loads:
            out[nz] += ricker(t0 + k * dt, f0) * bv
        out *= im
        return out

    snaps = {}
    trace = []
    rec = None if receivers is None else np.asarray(receivers)
    if resume is not None:
        u_prev, u, k = resume["u_prev"], resume["u"], resume["k"]
        a = np.empty(prob.ndof)
        return _cdm_loop(k, nsteps, u_prev, u, a, accel, dt, checkpoints, snaps, rec, trace,
                         progress)
    if 0 in checkpoints:
        snaps[0] = u.copy()
    if rec is not None:
        trace.append(rec @ u)
    if nsteps == 0:
        return dict(u=u, u_prev=u - dt * v, k=0, snapshots=snaps,
                    trace=None if rec is None else np.array(trace))
    a = accel(0, u, np.empty(prob.ndof))
    u_prev = u
    u = u + dt * v + 0.5 * dt * dt * a
    k = 1
    if k in checkpoints:
        snaps[k] = u.copy()
    if rec is not None:
        trace.append(rec @ u)
    if progress:
        progress(k)
    return _cdm_loop(k, nsteps, u_prev.copy(), u, a, accel, dt, checkpoints, snaps, rec, trace,
                     progress)


def _cdm_loop(k, nsteps, u_prev, u, a, accel, dt, checkpoints, snaps, rec, trace, progress):
    """Steps k -> nsteps of eq. cdm from (u_{k-1}, u_k)."""
    while k < nsteps:
        accel(k, u, a)
        # u_{k+1} = 2 u_k - u_{k-1} + dt^2 a, stored in the array of u_{k-1}
        np.subtract(u, u_prev, out=u_prev)
        u_prev += u
        a *= dt * dt
        u_prev += a
        u_prev, u = u, u_prev
        k += 1
        if k in checkpoints:
            snaps[k] = u.copy()
        if rec is not None:
            trace.append(rec @ u)
        if progress:
            progress(k)
    return dict(u=u, u_prev=u_prev, k=k, snapshots=snaps,
                trace=None if rec is None else np.array(trace))


def energy(disc, u_k, u_k1, dt):
    """Discrete energy of the central difference scheme between steps k and k+1:
    E_{k+1/2} = 1/2 v^T M v + 1/2 u_{k+1}^T K u_k with v = (u_{k+1} - u_k)/dt.
    With K symmetric and F = 0 it is exactly conserved by eq. cdm; with a load,
    E_{k+1/2} - E_{k-1/2} = 1/2 F_k^T (u_{k+1} - u_{k-1})."""
    prob = disc.prob
    m = np.tile(disc.mass, prob.ncomp)
    v = (u_k1 - u_k) / dt
    return 0.5 * float(v @ (m * v)) + 0.5 * float(u_k1 @ apply_K(disc, u_k))
