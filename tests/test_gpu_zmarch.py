"""GPU tests of the 3-D z-marching step kernel (zmarch.h).

The kernel takes the tile kernel's arithmetic operation for operation (the same K_ref
fragments and k order on the matrix cores, the same per-node summation order, the same
update), so on the same inputs its states must equal the tile kernel's bit for bit; its
oracle parity on a one-chunk grid runs with every other configuration in
tests/test_gpu_parity.py.  Here the grids have several z chunks (the last one ragged),
ragged x-y tiles, a source whose cell straddles a chunk boundary and several right-hand
sides; batched runs and graph replays with the kernel equal single runs.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

H = 0.02
# first source: its cell's top node plane (z = 0.32) is the first plane of the second
# 16-layer chunk
SRC = [dict(x=(0.05, 0.05, 0.319), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0),
       dict(x=(0.15, 0.11, 0.61), dir=(0.0, 0.6, 0.8), f0=14.0, amp=-0.5)]


def _cfg(n, seed):
    rng = np.random.default_rng(seed)
    hi = tuple(H * k for k in n)
    cc = rng.uniform(0.0, 1.0, (12, 3)) * np.array(hi)
    rr = rng.uniform(0.02, 0.05, 12)
    keep = np.ones(len(rr), dtype=bool)
    for s in SRC:
        keep &= np.linalg.norm(cc - np.array(s["x"]), axis=1) > rr + 0.02
    return workloads._base(3, n, 2, cc[keep], rr[keep], ncomp=3, tree_depth=2, hi=hi)


def _zconfigs(s):
    return [i for i, c in enumerate(s.tile_configs()) if "zmarch_kernel" in c["kernel"]]


def _run(s, i, dt, nsteps, nrhs=2):
    import torch
    s.select_tile(i)
    u, d = s.zeros(nrhs), s.zeros(nrhs)
    s.step(u, d, SRC[:nrhs], dt, nsteps, start=True)
    torch.cuda.synchronize()
    return u.cpu().numpy().copy(), d.cpu().numpy().copy()


@pytest.fixture(scope="module")
def tall():
    from paper_2501_19013_amd.solver import Solver
    cfg = _cfg((10, 9, 37), 41)
    s = Solver(cfg, precision="fp32")
    dt = 0.9 * s.critical_dt()
    yield cfg, s, dt
    s.close()


def test_zmarch_equals_tile_kernel(tall):
    """Every z-marching configuration (8x8 and 8x4 tiles, 16 and 32 layers per item: three
    and two chunks over 37 layers) against the default tile kernel, u and d bit for bit,
    two right-hand sides, 23 steps from the Newmark start-up."""
    cfg, s, dt = tall
    zc = _zconfigs(s)
    assert len(zc) >= 2
    u0, d0 = _run(s, 0, dt, 23)
    assert np.abs(u0).max() > 0
    for i in zc:
        u, d = _run(s, i, dt, 23)
        assert np.array_equal(u, u0), (i, float(np.abs(u - u0).max()))
        assert np.array_equal(d, d0), i
    s.select_tile(0)


def test_zmarch_single_rhs_and_odd_step_count(tall):
    cfg, s, dt = tall
    zc = _zconfigs(s)
    u0, d0 = _run(s, 0, dt, 8, nrhs=1)
    for i in zc:
        u, d = _run(s, i, dt, 8, nrhs=1)
        assert np.array_equal(u, u0), i
        assert np.array_equal(d, d0), i
    s.select_tile(0)


def test_zmarch_batched_and_graph_equal_alone():
    """Two 3-D elastic problems of different shapes advanced together with a z-marching
    configuration chosen on the first (the owner), eagerly and by graph replay, equal each
    problem run alone with that configuration."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    stream = torch.cuda.Stream()
    probs = []
    for n, seed, nsteps in (((10, 9, 37), 42, 19), ((17, 7, 32), 43, 26)):
        s = Solver(_cfg(n, seed), precision="fp32", stream=stream)
        probs.append((s, 0.9 * s.critical_dt(), nsteps))
    zc = _zconfigs(probs[0][0])
    assert zc
    for i in zc:
        alone = [_run(s, i, dt, n)[0] for s, dt, n in probs]
        for s, _, _ in probs:
            s.select_tile(i)
        for use_graph in (False, True, True):
            states = [(s.zeros(2), s.zeros(2)) for s, _, _ in probs]
            with torch.cuda.stream(stream):
                fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC, dt=dt, nsteps=n, start=1)
                         for (s, dt, n), (u, d) in zip(probs, states)], graph=use_graph)
            torch.cuda.synchronize()
            for (u, _), ref in zip(states, alone):
                assert np.array_equal(u.cpu().numpy(), ref), (i, use_graph)
    for s, _, _ in probs:
        s.close()
