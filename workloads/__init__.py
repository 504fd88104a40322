"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module draws random geometry and builds plain configuration dictionaries.  It
holds none of the method's arithmetic (no basis functions, quadrature, matrices or
time stepping): only the void fields, source positions and sizes that both the
oracle and the HIP path consume bit for bit.

Workloads (immersed-boundary wave problems on a Cartesian box, Sec. 2.1-2.2 of the
paper; the paper's own benchmark is a rotated cube, Sec. 3.1, which these synthetic
void fields stand in for):

* ``c1``: 2-D scalar wave on [0,1]^2 with one circular hole r=0.25 at the centre,
  16x16 cells, p=3, quadtree depth 3, eps=1e-4, Ricker f0=10 at (0.1,0.1), 500 steps.
* ``c2``: 2-D scalar wave on [0,1]^2 with 40 random circular voids (r ~ U(0.01,0.05),
  seed 2), 512x512 cells, p=4 (about 4.2M DOF), 2000 steps.
* ``c3``: 3-D linear elastodynamics on the unit cube with a random spherical pore
  field (porosity 0.2, r ~ U(0.02,0.06), seed 3), 96^3 cells, p=2, E=1, nu=0.3.
* ``c4``: as c3 at 64^3 cells, p=3, 16 sources.
* ``c5``: a stream of 256 requests with Poisson arrivals (seed 5).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "circle_hole", "random_circles", "random_spheres", "config", "scaled_config",
    "request_stream", "CONFIG_NAMES", "cardan_rotation", "rotated_cube", "cube_point",
    "cube_observers",
]

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


def circle_hole(center=(0.5, 0.5), radius=0.25):
    """One circular void (c1)."""
    return np.array([center], dtype=np.float64), np.array([radius], dtype=np.float64)


def random_circles(seed=2, count=40, rmin=0.01, rmax=0.05, lo=0.0, hi=1.0,
                   keep_clear=((0.1, 0.1),)):
    """``count`` circles with r ~ U(rmin, rmax) and centres ~ U(lo+r, hi-r)^2.

    A draw whose disc contains any point of ``keep_clear`` (sources, receivers) is
    rejected and drawn again; overlaps between circles are allowed.
    """
    rng = np.random.default_rng(seed)
    keep = np.asarray(keep_clear, dtype=np.float64).reshape(-1, 2)
    centers, radii = [], []
    while len(radii) < count:
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(lo + r, hi - r, 2)
        if keep.size and np.any(np.linalg.norm(keep - c, axis=1) <= r):
            continue
        centers.append(c)
        radii.append(r)
    return np.array(centers, dtype=np.float64), np.array(radii, dtype=np.float64)


def random_spheres(seed=3, porosity=0.2, rmin=0.02, rmax=0.06, n_probe=200000,
                   keep_clear=((0.1, 0.1, 0.1),), max_spheres=100000):
    """Spheres with r ~ U(rmin, rmax), centres ~ U[0,1]^3, added until a Monte-Carlo
    estimate of the void fraction (``n_probe`` uniform points) reaches ``porosity``.

    A draw whose ball contains a point of ``keep_clear`` is rejected.
    """
    rng = np.random.default_rng(seed)
    probe = rng.random((n_probe, 3))
    inside = np.zeros(n_probe, dtype=bool)
    keep = np.asarray(keep_clear, dtype=np.float64).reshape(-1, 3)
    centers, radii = [], []
    while len(radii) < max_spheres:
        r = rng.uniform(rmin, rmax)
        c = rng.random(3)
        if keep.size and np.any(np.linalg.norm(keep - c, axis=1) <= r):
            continue
        centers.append(c)
        radii.append(r)
        inside |= np.sum((probe - c) ** 2, axis=1) < r * r
        if inside.mean() >= porosity:
            break
    return np.array(centers, dtype=np.float64), np.array(radii, dtype=np.float64)


def _base(dim, ncells, p, centers, radii, **kw):
    cfg = dict(
        dim=dim, ncomp=1, ncells=tuple(int(n) for n in ncells),
        lo=(0.0,) * dim, hi=(1.0,) * dim, p=int(p), tree_depth=3,
        void_center=np.asarray(centers, dtype=np.float64).reshape(-1, dim),
        void_radius=np.asarray(radii, dtype=np.float64).reshape(-1),
        alpha=1e-12, rho=1.0, c=1.0, E=1.0, nu=0.3,
        eps=1e-4, f_lambda=1e-4,
        sources=[dict(x=(0.1,) * dim, dir=(1.0, 0.0, 0.0)[:max(dim, 1)], f0=10.0, amp=1.0)],
        nsteps=500, dt_factor=0.9, dt_max=np.inf,
    )
    cfg.update(kw)
    return cfg


def config(name):
    """Full-size configuration dictionary for workload ``name`` (c1..c4)."""
    if name == "c1":
        cc, rr = circle_hole()
        return _base(2, (16, 16), 3, cc, rr, nsteps=500)
    if name == "c2":
        cc, rr = random_circles(seed=2)
        return _base(2, (512, 512), 4, cc, rr, nsteps=2000)
    if name == "c3":
        cc, rr = random_spheres(seed=3)
        return _base(3, (96, 96, 96), 2, cc, rr, ncomp=3, nsteps=1000)
    if name == "c4":
        cc, rr = random_spheres(seed=3)
        src = [dict(x=(x, y, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0)
               for y in (0.2, 0.4, 0.6, 0.8) for x in (0.2, 0.4, 0.6, 0.8)]
        return _base(3, (64, 64, 64), 3, cc, rr, ncomp=3, nsteps=1000, sources=src,
                     eps=0.0)
    raise KeyError(name)


def scaled_config(dim, n, p, seed, nvoids=None, ncomp=1, porosity=None,
                  rmin=None, rmax=None, nsteps=100, depth=3, **kw):
    """A smaller problem of the same kind as c2 (dim=2) or c3 (dim=3), for parity tests.

    ``n`` cells per direction; void radii are those of the full-size workload unless
    given, so the cut-cell structure per unit area/volume matches it.
    """
    if dim == 2:
        cc, rr = random_circles(seed=seed, count=40 if nvoids is None else nvoids,
                                rmin=0.01 if rmin is None else rmin,
                                rmax=0.05 if rmax is None else rmax)
    else:
        cc, rr = random_spheres(seed=seed, porosity=0.2 if porosity is None else porosity,
                                rmin=0.02 if rmin is None else rmin,
                                rmax=0.06 if rmax is None else rmax, n_probe=50000)
    return _base(dim, (n,) * dim, p, cc, rr, ncomp=ncomp, nsteps=nsteps,
                 tree_depth=depth, **kw)


def cardan_rotation(phi, theta, psi):
    """Rotation matrix T = R_z(psi) R_y(theta) R_x(phi) of Cardan angles in degrees
    (columns: the rotated frame's axes in global coordinates).  The paper names the
    angles but not their order; this order reproduces most of its printed DOF counts."""
    a, b, g = np.deg2rad([phi, theta, psi])
    rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    rz = np.array([[np.cos(g), -np.sin(g), 0], [np.sin(g), np.cos(g), 0], [0, 0, 1]])
    return rz @ ry @ rx


def rotated_cube(n, p, l_p=0.3, l_e=0.5, angles=(10.0, 10.0, 10.0), **kw):
    """The paper's benchmark geometry (Sec. 3.1): a cube of edge l_p rotated by the Cardan
    angles about the common centre of an embedding cube of edge l_e, here
    [-l_e/2, l_e/2]^3 with n cells per direction, GLL degree p, scalar wave, no voids.
    Sources and observers are given in the cube's local frame (origin at its centre)
    and mapped to global coordinates with cube_point."""
    T = cardan_rotation(*angles)
    cfg = _base(3, (n, n, n), p, np.zeros((0, 3)), np.zeros(0),
                lo=(-l_e / 2,) * 3, hi=(l_e / 2,) * 3, **kw)
    cfg["cube"] = dict(center=np.zeros(3), half=l_p / 2, rot=T)
    cfg["l_p"] = l_p
    cfg["sources"] = [dict(x=tuple(cube_point(cfg, (-l_p / 2, 0.0, 0.0))), f0=10.0, amp=1.0)]
    return cfg


def cube_point(cfg, x_local):
    """Global coordinates x = c + T x' of a point given in the cube's frame."""
    c = cfg["cube"]
    return np.asarray(c["center"]) + np.asarray(c["rot"]) @ np.asarray(x_local, dtype=np.float64)


def cube_observers(cfg):
    """The 11 observer points of Table observer_locations (source, centre, face centre, 4
    edge centres, 4 corners), given there with the origin at a cube corner (x' in
    [0, l]^3), in global coordinates."""
    l = cfg["l_p"]
    h = l / 2
    pts = [(0.0, h, h), (h, h, h), (l, h, h)]
    pts += [(h, h + sy * h, h + sz * h) for sy in (-1, 1) for sz in (-1, 1)]
    pts += [(l, h + sy * h, h + sz * h) for sy in (-1, 1) for sz in (-1, 1)]
    return np.array([cube_point(cfg, np.array(x) - h) for x in pts])


def request_stream(seed=5, count=256, rate=None):
    """Serving workload (c5): ``count`` requests with Poisson arrivals.

    Each request is a 2-D or 3-D scalar immersed-void problem: side uniform on
    [64, 1024] (2-D) or [16, 96] (3-D) cells, p in {2,3,4}, steps in [200, 2000],
    void seed 1000+id.  ``rate`` (requests/s) sets the exponential inter-arrival
    times; ``None`` gives arrival time 0 for all (closed-loop).
    """
    rng = np.random.default_rng(seed)
    arr = np.random.default_rng([seed, 1])  # arrivals apart: the requests do not depend on rate
    reqs = []
    t = 0.0
    for i in range(count):
        dim = 2 if rng.random() < 0.5 else 3
        side = int(rng.integers(64, 1025)) if dim == 2 else int(rng.integers(16, 97))
        p = int(rng.integers(2, 5))
        steps = int(rng.integers(200, 2001))
        if rate is not None:
            t += arr.exponential(1.0 / rate)
        reqs.append(dict(id=i, dim=dim, n=side, p=p, nsteps=steps, void_seed=1000 + i,
                         arrival=t))
    return reqs
