"""GPU tests of batched runs (fcw_run): several 2-D problems of one kind, many
right-hand sides, different sizes and step counts in shared launches; a batched result
must equal the same problem run alone bit for bit (same kernels, same per-node
summation order), and HIP-graph replays must equal eager runs."""
import numpy as np
import pytest

import workloads
from oracle import problem, timestep

pytestmark = pytest.mark.gpu


def _cfg(n, seed, p=3, nvoids=10):
    cfg = workloads.config("c2")
    cc, rr = workloads.random_circles(seed=seed, count=nvoids, rmin=0.02, rmax=0.08,
                                      keep_clear=((0.1, 0.1), (0.7, 0.3)))
    cfg.update(ncells=(n, n), p=p, void_center=cc, void_radius=rr)
    return cfg


SRC = [dict(x=(0.1, 0.1), f0=10.0, amp=1.0), dict(x=(0.7, 0.3), f0=14.0, amp=-0.5)]


@pytest.fixture(scope="module")
def problems():
    import torch
    from paper_2501_19013_amd.solver import Solver
    stream = torch.cuda.Stream()
    out = []
    for n, seed, nsteps in ((40, 21, 120), (64, 22, 97), (23, 23, 150)):
        cfg = _cfg(n, seed)
        s = Solver(cfg, precision="fp32", stream=stream)
        dtc = s.critical_dt()
        out.append((cfg, s, 0.9 * dtc, nsteps))
    return stream, out


def _alone(s, dt, nsteps):
    import torch
    u, d = s.zeros(2), s.zeros(2)
    s.step(u, d, SRC, dt, nsteps, start=True)
    torch.cuda.synchronize()
    return u.cpu().numpy().copy()


def test_batched_equals_alone(problems):
    import torch
    from paper_2501_19013_amd import fcw
    stream, probs = problems
    alone = [_alone(s, dt, n) for _, s, dt, n in probs]
    states = [(s.zeros(2), s.zeros(2)) for _, s, _, _ in probs]
    with torch.cuda.stream(stream):
        fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC, t0=0.0, dt=dt, nsteps=n, start=1)
                 for (_, s, dt, n), (u, d) in zip(probs, states)])
    torch.cuda.synchronize()
    for (u, _), ref in zip(states, alone):
        assert np.array_equal(u.cpu().numpy(), ref)


def test_batched_matches_oracle(problems):
    import torch
    from paper_2501_19013_amd import fcw
    stream, probs = problems
    cfg, s, dt, n = probs[2]
    u, d = s.zeros(2), s.zeros(2)
    with torch.cuda.stream(stream):
        fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC, dt=dt, nsteps=n, start=1)])
    torch.cuda.synchronize()
    disc = problem.build(problem.Problem.from_config(cfg))
    for r in range(2):
        ref = timestep.cdm(disc, dt, n, sources=[SRC[r]])["u"]
        got = u[r].double().cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4


def test_graph_replays_equal_eager(problems):
    import torch
    from paper_2501_19013_amd import fcw
    stream, probs = problems
    q = 40  # a quantum of steps per call
    eager = [(s.zeros(2), s.zeros(2)) for _, s, _, _ in probs]
    graph = [(s.zeros(2), s.zeros(2)) for _, s, _, _ in probs]
    for k in range(4):   # 4 quanta: one capture, three replays
        for st, use_graph in ((eager, False), (graph, True)):
            with torch.cuda.stream(stream):
                fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC, t0=k * q * dt, dt=dt,
                              nsteps=q, start=int(k == 0))
                         for (_, s, dt, _), (u, d) in zip(probs, st)], graph=use_graph)
            # the program's own eager work and a synchronisation between replays
            torch.cuda.synchronize()
            _ = (eager[0][0] * 2.0).sum().item()
        for (ue, _), (ug, _) in zip(eager, graph):
            assert np.array_equal(ue.cpu().numpy(), ug.cpu().numpy()), k


def test_finished_problem_drops_out(problems):
    # a problem with fewer steps in the batch stops at its own count
    import torch
    from paper_2501_19013_amd import fcw
    stream, probs = problems
    (_, s0, dt0, _), (_, s1, dt1, _) = probs[0], probs[1]
    ref0 = _alone(s0, dt0, 31)
    ref1 = _alone(s1, dt1, 80)
    a, b = (s0.zeros(2), s0.zeros(2)), (s1.zeros(2), s1.zeros(2))
    with torch.cuda.stream(stream):
        fcw.run([dict(ctx=s0.ctx, nrhs=2, u=a[0], d=a[1], sources=SRC, dt=dt0, nsteps=31, start=1),
                 dict(ctx=s1.ctx, nrhs=2, u=b[0], d=b[1], sources=SRC, dt=dt1, nsteps=80, start=1)])
    torch.cuda.synchronize()
    assert np.array_equal(a[0].cpu().numpy(), ref0)
    assert np.array_equal(b[0].cpu().numpy(), ref1)


def test_graph_cache_follows_member_layout():
    # A graph captured for one work-list layout must not be replayed for another with
    # the same item and step counts: five void-free members (one 64^2, four 32^2), then
    # two 64^2 members, 64 items each with tile (21, 8); the second list fits the first's
    # buffer, so only the member count tells the layouts apart.
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    stream = torch.cuda.Stream()
    src = [dict(x=(0.13, 0.21), f0=10.0, amp=1.0)]

    def solver(n):
        cfg = workloads._base(2, (n, n), 3, np.zeros((0, 2)), np.zeros(0))
        s = Solver(cfg, precision="fp32", stream=stream)
        tiles = s.tile_configs()
        i = next(k for k, t in enumerate(tiles) if tuple(t["tile"][:2]) == (21, 8))
        s.select_tile(i)
        return s

    big = [solver(64), solver(64)]
    small = [solver(32) for _ in range(4)]
    dt = 1e-3
    nsteps = 12

    def run(members, use_graph):
        st = [(s.zeros(1), s.zeros(1)) for s in members]
        with torch.cuda.stream(stream):
            fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=src, dt=dt, nsteps=nsteps,
                          start=1) for s, (u, d) in zip(members, st)], graph=use_graph)
        torch.cuda.synchronize()
        return [u.cpu().numpy().copy() for u, _ in st]

    first = [big[0]] + small
    for a, b in zip(run(first, True), run(first, False)):
        assert np.array_equal(a, b)
    second = [big[0], big[1]]
    for a, b in zip(run(second, True), run(second, False)):
        assert np.array_equal(a, b)
    for s in big + small:
        s.close()


# ---------------------------------------------------------------- 3-D problems of one kind

SRC3 = [dict(x=(0.1, 0.1, 0.1), dir=(1.0, 0.0, 0.0), f0=10.0, amp=1.0),
        dict(x=(0.62, 0.33, 0.41), dir=(0.0, 0.6, 0.8), f0=14.0, amp=-0.5)]


def _cfg3(n, seed, hi=None):
    cc, rr = workloads.random_spheres(seed=seed, porosity=0.12, rmin=0.06, rmax=0.12,
                                      n_probe=20000, keep_clear=tuple(q["x"] for q in SRC3))
    kw = {} if hi is None else dict(hi=hi)
    return workloads._base(3, n, 2, cc, rr, ncomp=3, tree_depth=2, **kw)


@pytest.fixture(scope="module")
def problems3d():
    import torch
    from paper_2501_19013_amd.solver import Solver
    stream = torch.cuda.Stream()
    out = []
    for n, seed, nsteps, hi in (((6, 6, 6), 31, 57, None), ((8, 7, 5), 32, 40, (0.8, 0.7, 0.5)),
                                ((5, 5, 5), 33, 73, None)):
        cfg = _cfg3(n, seed, hi)
        s = Solver(cfg, precision="fp32", stream=stream)
        out.append((cfg, s, 0.9 * s.critical_dt(), nsteps))
    return stream, out


def _alone3(s, dt, nsteps):
    import torch
    u, d = s.zeros(2), s.zeros(2)
    s.step(u, d, SRC3, dt, nsteps, start=True)
    torch.cuda.synchronize()
    return u.cpu().numpy().copy()


def test_3d_batched_equals_alone(problems3d):
    """Three 3-D elastic problems of different sizes and step counts in shared launches
    equal each problem run alone, bit for bit (same kernel, same per-node order)."""
    import torch
    from paper_2501_19013_amd import fcw
    stream, probs = problems3d
    alone = [_alone3(s, dt, n) for _, s, dt, n in probs]
    states = [(s.zeros(2), s.zeros(2)) for _, s, _, _ in probs]
    with torch.cuda.stream(stream):
        fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC3, dt=dt, nsteps=n, start=1)
                 for (_, s, dt, n), (u, d) in zip(probs, states)])
    torch.cuda.synchronize()
    for (u, _), ref in zip(states, alone):
        assert np.abs(ref).max() > 0
        assert np.array_equal(u.cpu().numpy(), ref)


def test_3d_batched_matches_oracle(problems3d):
    import torch
    from paper_2501_19013_amd import fcw
    stream, probs = problems3d
    (cfg, s, dt, n), (_, s2, dt2, n2) = probs[1], probs[0]
    u, d = s.zeros(2), s.zeros(2)
    u2, d2 = s2.zeros(2), s2.zeros(2)
    with torch.cuda.stream(stream):
        fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC3, dt=dt, nsteps=n, start=1),
                 dict(ctx=s2.ctx, nrhs=2, u=u2, d=d2, sources=SRC3, dt=dt2, nsteps=n2, start=1)])
    torch.cuda.synchronize()
    disc = problem.build(problem.Problem.from_config(cfg))
    for r in range(2):
        ref = timestep.cdm(disc, dt, n, sources=[SRC3[r]])["u"]
        got = u[r].double().cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4


def test_3d_graph_replays_equal_eager(problems3d):
    import torch
    from paper_2501_19013_amd import fcw
    stream, probs = problems3d
    q = 15
    eager = [(s.zeros(2), s.zeros(2)) for _, s, _, _ in probs]
    graph = [(s.zeros(2), s.zeros(2)) for _, s, _, _ in probs]
    for k in range(3):
        for st, use_graph in ((eager, False), (graph, True)):
            with torch.cuda.stream(stream):
                fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC3, t0=k * q * dt, dt=dt,
                              nsteps=q, start=int(k == 0))
                         for (_, s, dt, _), (u, d) in zip(probs, st)], graph=use_graph)
            torch.cuda.synchronize()
            _ = (eager[0][0] * 2.0).sum().item()
        for (ue, _), (ug, _) in zip(eager, graph):
            assert np.array_equal(ue.cpu().numpy(), ug.cpu().numpy()), k
