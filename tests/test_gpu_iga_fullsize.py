"""IGA-FCM parity at the full size of its benchmark leg (the c2 void field, 512^2 cells,
B-splines p = 4, 516^2 DOFs), on sampled DOFs the oracle computes one by one (the whole
problem is too large for the numpy oracle), in the launch configuration the benchmark
times (FP32 steps through fcw_iga_step):

* the row-sum lumped mass at the samples (FP64), from the oracle's own element matrices
  of the cells around each sample (the cells' classes bit-exact first);
* the FP64 stiffness action of a seeded random state at the samples;
* one FP32 step from a seeded random state (u_k, d_k) with the point source active:
  d_{k+1} = d_k + dt^2 m^{-1} (F_k - K u_k) and u_{k+1} = u_k + d_{k+1} at the samples.

Samples: the DOFs of the source cell, of cut cells, of cells at the box's faces and
corners (the boundary position classes of the open knot vectors), and random DOFs.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import geometry, iga
from oracle.problem import Problem, ricker

pytestmark = pytest.mark.gpu


class _IgaCells:
    """Oracle element matrices of single cells, on demand."""

    def __init__(self, prob, cls):
        self.prob, self.cls, self.kv, self.cache = prob, cls, iga.knots(prob), {}

    def get(self, cell):
        if cell not in self.cache:
            c = self.cls[cell]
            km = None if c == geometry.OUT else iga.cell_matrices(self.prob, self.kv, cell, c)
            self.cache[cell] = km
        return self.cache[cell]


def _cells_of_dof(prob, dof):
    """Cells supporting a DOF (lexicographic, x fastest) and the DOF's local index in each."""
    nb = [n + prob.p for n in prob.ncells]
    i = [dof % nb[0], dof // nb[0]]
    out = []
    for cy in range(max(i[1] - prob.p, 0), min(i[1], prob.ncells[1] - 1) + 1):
        for cx in range(max(i[0] - prob.p, 0), min(i[0], prob.ncells[0] - 1) + 1):
            out.append((cx + prob.ncells[0] * cy, (i[0] - cx) + (prob.p + 1) * (i[1] - cy)))
    return out


def test_iga_full_size_samples():
    import torch
    from paper_2501_19013_amd import fcw
    cfg = workloads.config("c2")
    prob = Problem.from_config(cfg)
    ctx = fcw.assemble_cells(cfg, precision="fp32")
    g = fcw.iga_create(ctx)
    try:
        info = fcw.iga_query(g)
        nb0 = 512 + prob.p
        n = info["ndof"]
        assert n == nb0 * nb0
        # classes: the device's (after dropping all-void cut cells) against the oracle's
        cls = fcw.export(ctx, 0).astype(np.int8)
        ocls = geometry.classify_cells(prob)
        diff = np.flatnonzero(cls != ocls)
        assert np.all((ocls[diff] == geometry.CUT) & (cls[diff] == geometry.OUT))
        cells = _IgaCells(prob, ocls.copy())
        rng = np.random.default_rng(17)
        samples = set(rng.integers(0, n, 120).tolist())
        src = cfg["sources"][0]
        cs = [min(max(int(math.floor((src["x"][k] - prob.lo[k]) / prob.h)), 0), 511)
              for k in range(2)]
        for jy in range(prob.p + 1):
            for jx in range(prob.p + 1):
                samples.add((cs[0] + jx) + nb0 * (cs[1] + jy))
        cut = np.flatnonzero(ocls == geometry.CUT)
        for cell in rng.choice(cut, 12, replace=False):
            cx, cy = int(cell) % 512, int(cell) // 512
            samples.update([(cx + 1) + nb0 * (cy + 2), (cx + 3) + nb0 * (cy + 1)])
        for dof in [0, 1, nb0 + 2, nb0 - 1, 3 * nb0 - 2, n - 1, n - nb0, n - 2 * nb0 + 3,
                    nb0 * 200, nb0 * 300 + nb0 - 3]:
            samples.add(dof)
        samples = np.array(sorted(samples))
        # oracle cells around the samples; a dropped cut cell must be OUT on the device
        for dof in samples:
            for cell, _ in _cells_of_dof(prob, int(dof)):
                if cells.get(cell) is None and ocls[cell] == geometry.CUT:
                    cells.cls[cell] = geometry.OUT
                assert cls[cell] == cells.cls[cell], cell
        mass = fcw.iga_export(g, fcw.FCW_IGA_ARR_MASS)
        m_ref = np.zeros(len(samples))
        for s, dof in enumerate(samples):
            for cell, loc in _cells_of_dof(prob, int(dof)):
                km = cells.get(cell)
                if km is not None:
                    m_ref[s] += km[1][loc].sum()
        np.testing.assert_allclose(mass[samples], m_ref, rtol=1e-11, atol=1e-14 * m_ref.max())

        table = iga.cell_dof_table(prob)

        def k_action(u, dof):
            acc = 0.0
            for cell, loc in _cells_of_dof(prob, int(dof)):
                km = cells.get(cell)
                if km is not None:
                    acc += km[0][loc] @ u[table[cell]]
            return acc

        # FP64 stiffness action of a seeded state (through an FP64 context of the same cells)
        u0 = rng.standard_normal(n)
        ctx64 = fcw.assemble_cells(cfg, precision="fp64")
        g64 = fcw.iga_create(ctx64)
        try:
            ud = torch.tensor(u0[None, :], device="cuda")
            rd = torch.zeros_like(ud)
            fcw.iga_apply_stiffness(g64, 1, ud, rd)
            torch.cuda.synchronize()
            r = rd[0].cpu().numpy()
        finally:
            fcw.iga_destroy(g64)
            fcw.destroy(ctx64)
        r_ref = np.array([k_action(u0, d) for d in samples])
        np.testing.assert_allclose(r[samples], r_ref, atol=1e-10 * np.abs(r_ref).max())

        # one FP32 step of the benchmark's launch configuration, source active
        u0 = (0.01 * rng.standard_normal(n)).astype(np.float32)
        d0 = (1e-4 * rng.standard_normal(n)).astype(np.float32)
        u0[mass == 0] = 0.0
        d0[mass == 0] = 0.0
        dt = 9.0e-4
        t0 = 0.08  # the Ricker pulse is near its peak
        uu = torch.tensor(u0[None, :], device="cuda")
        dd = torch.tensor(d0[None, :], device="cuda")
        fcw.iga_step(g, 1, uu, dd, [src], t0, dt, 1, 0)
        torch.cuda.synchronize()
        u1, d1 = uu[0].cpu().numpy(), dd[0].cpu().numpy()
        scell, sval = iga.source_values(prob, src["x"])
        b = np.zeros(n)
        b[table[scell]] = prob.rho * src.get("amp", 1.0) * sval
        ft = ricker(t0, src["f0"])
        u064, d064 = u0.astype(np.float64), d0.astype(np.float64)
        d_ref = np.array([d064[dof] + dt * dt / m_ref[s] * (ft * b[dof] - k_action(u064, dof))
                          if m_ref[s] > 0 else d064[dof] for s, dof in enumerate(samples)])
        u_ref = u064[samples] + d_ref
        assert np.abs(b[samples]).max() > 0
        np.testing.assert_allclose(d1[samples], d_ref, atol=1e-4 * np.abs(d_ref).max())
        np.testing.assert_allclose(u1[samples], u_ref, atol=1e-5 * np.abs(u_ref).max())
    finally:
        fcw.iga_destroy(g)
        fcw.destroy(ctx)
