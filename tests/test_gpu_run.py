"""GPU tests of fcw_run's observation and control: receiver traces against the oracle's
observer rows (Sec. 3.2), the step size rule dt = min(0.9 dt_crit, dt_max) (Sec. 3.3),
growth detection above the critical step (Sec. 2.3), the discrete energy after the run,
and the per-problem results.

Bars: FP64 traces within 1e-10 of the largest trace value (same finite recurrence, other
summation order); FP32 traces within 1e-4; integer outcomes (status, steps) exact."""
import numpy as np
import pytest

import workloads
from oracle import problem, timestep

pytestmark = pytest.mark.gpu

REC2 = [(0.83, 0.27), (0.31, 0.74), (0.9, 0.9)]
SRC2 = [dict(x=(0.1, 0.1), f0=10.0, amp=1.0), dict(x=(0.7, 0.3), f0=14.0, amp=-0.5)]


@pytest.fixture(scope="module")
def c1():
    cfg = workloads.config("c1")
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = 0.9 * timestep.critical_dt(disc)
    return cfg, disc, dt


def _traces_buf(nrhs, nsteps, nrec, ncomp=1):
    import torch
    return torch.full((nrhs, nsteps + 1, nrec, ncomp), float("nan"), dtype=torch.float64,
                      device="cuda")


def _oracle_traces(disc, dt, nsteps, srcs, rec):
    R = problem.receiver_rows(disc, rec)
    return [timestep.cdm(disc, dt, nsteps, sources=[s], receivers=R)["trace"] for s in srcs]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_traces_match_oracle_2d(c1, precision, tol):
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, disc, dt = c1
    nsteps = 240
    s = Solver(cfg, precision=precision)
    u, d = s.zeros(2), s.zeros(2)
    tr = _traces_buf(2, nsteps, len(REC2))
    out = fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC2, dt=dt, nsteps=nsteps,
                        start=1, receivers=REC2, traces=tr)])
    torch.cuda.synchronize()
    assert out[0]["status"] == fcw.FCW_OK and out[0]["steps_done"] == nsteps
    got = tr.cpu().numpy()[..., 0]
    ref = _oracle_traces(disc, dt, nsteps, SRC2, REC2)
    for q in range(2):
        scale = np.abs(ref[q]).max()
        assert scale > 0
        assert np.abs(got[q] - ref[q]).max() <= tol * scale, (q, np.abs(got[q] - ref[q]).max())
    s.close()


def test_traces_match_oracle_3d_elastic():
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg = workloads.scaled_config(3, 4, 2, seed=4, ncomp=3, porosity=0.2)
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = 0.9 * timestep.critical_dt(disc)
    rec = [(0.8, 0.3, 0.55), (0.3, 0.3, 0.3)]
    rec = [x for x in rec if not np.any(np.linalg.norm(cfg["void_center"] - x, axis=1)
                                        < cfg["void_radius"])]
    assert rec
    nsteps = 90
    src = cfg["sources"]
    s = Solver(cfg, precision="fp64")
    u, d = s.zeros(1), s.zeros(1)
    tr = _traces_buf(1, nsteps, len(rec), 3)
    fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=src, dt=dt, nsteps=nsteps, start=1,
                  receivers=rec, traces=tr)])
    torch.cuda.synchronize()
    got = tr.cpu().numpy()[0].reshape(nsteps + 1, -1)
    ref = _oracle_traces(disc, dt, nsteps, src, rec)[0]
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(got - ref).max() <= 1e-10 * scale
    s.close()


def test_traces_in_a_batched_group_equal_alone(c1):
    """Two 2-D problems of one kind with receivers share launches; their traces equal the
    traces of each run alone, bit for bit, and the state equals the run without
    receivers."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, disc, dt = c1
    cfg2 = dict(cfg)
    cc, rr = workloads.random_circles(seed=41, count=6, rmin=0.03, rmax=0.08,
                                      keep_clear=((0.1, 0.1), (0.7, 0.3)) + tuple(REC2))
    cfg2.update(ncells=(24, 24), void_center=cc, void_radius=rr)
    probs = [(Solver(cfg, precision="fp64"), 150), (Solver(cfg2, precision="fp64"), 111)]
    dts = [dt, 0.9 * probs[1][0].critical_dt()]
    alone, plain = [], []
    for (s, n), h in zip(probs, dts):
        u, d = s.zeros(2), s.zeros(2)
        tr = _traces_buf(2, n, len(REC2))
        fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC2, dt=h, nsteps=n, start=1,
                      receivers=REC2, traces=tr)])
        u2, d2 = s.zeros(2), s.zeros(2)
        s.step(u2, d2, SRC2, h, n, start=True)
        torch.cuda.synchronize()
        alone.append((u.cpu().numpy(), tr.cpu().numpy()))
        plain.append(u2.cpu().numpy())
    states = [(s.zeros(2), s.zeros(2), _traces_buf(2, n, len(REC2))) for s, n in probs]
    fcw.run([dict(ctx=s.ctx, nrhs=2, u=u, d=d, sources=SRC2, dt=h, nsteps=n, start=1,
                  receivers=REC2, traces=tr)
             for (s, n), h, (u, d, tr) in zip(probs, dts, states)])
    torch.cuda.synchronize()
    for (u, d, tr), (ua, tra), up in zip(states, alone, plain):
        assert np.array_equal(u.cpu().numpy(), ua)
        assert np.array_equal(ua, up)
        assert np.array_equal(tr.cpu().numpy(), tra)
        assert not np.isnan(tra).any()
    for s, _ in probs:
        s.close()


def test_step_size_rule_and_results(c1):
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, _, _ = c1
    s = Solver(cfg, precision="fp64")
    dtc = s.critical_dt()
    for dt_max, want in ((0.0, 0.9 * dtc), (1.0, 0.9 * dtc), (0.5 * dtc, 0.5 * dtc)):
        u, d = s.zeros(1), s.zeros(1)
        out = fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=SRC2[:1], dt=0.0,
                            dt_max=dt_max, nsteps=7, start=1)])
        assert out[0]["dt_used"] == want
        assert out[0]["steps_done"] == 7 and out[0]["status"] == fcw.FCW_OK
        # the same run with that step given explicitly
        u2, d2 = s.zeros(1), s.zeros(1)
        s.step(u2, d2, SRC2[:1], want, 7, start=True)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), u2.cpu().numpy())
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_growth_detection(c1, precision):
    """Above the critical step the highest mode grows and the problem is stopped with
    FCW_E_UNSTABLE; a problem at 0.9 dt_crit in the same run finishes its steps."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, _, _ = c1
    nsteps = 3000
    a = Solver(cfg, precision=precision)
    b = Solver(cfg, precision=precision)
    dtc = a.critical_dt()
    b.critical_dt()
    ua, da = a.zeros(1), a.zeros(1)
    ub, db = b.zeros(1), b.zeros(1)
    items = [dict(ctx=a.ctx, nrhs=1, u=ua, d=da, sources=SRC2[:1], dt=1.05 * dtc,
                  nsteps=nsteps, start=1, check_every=50),
             dict(ctx=b.ctx, nrhs=1, u=ub, d=db, sources=SRC2[:1], dt=0.9 * dtc,
                  nsteps=nsteps, start=1, check_every=50, energy=True)]
    with pytest.raises(fcw.FcwError) as e:
        fcw.run(items)
    assert e.value.status == fcw.FCW_E_UNSTABLE
    out = fcw.run([dict(it, u=x, d=y) for it, x, y in
                   zip(items, (a.zeros(1), b.zeros(1)), (a.zeros(1), b.zeros(1)))],
                  raise_unstable=False)
    torch.cuda.synchronize()
    assert out[0]["status"] == fcw.FCW_E_UNSTABLE
    assert 0 < out[0]["steps_done"] < nsteps and out[0]["steps_done"] % 50 == 0
    assert out[1]["status"] == fcw.FCW_OK and out[1]["steps_done"] == nsteps
    assert 0 < out[1]["growth"] < 1e6
    assert np.isfinite(ub.cpu().numpy()).all()
    a.close()
    b.close()


@pytest.mark.parametrize("check_every", [3, 10, 50])
def test_no_false_alarm_during_the_source_onset(c1, check_every):
    """A Ricker pulse switched on from rest grows by e^24 in amplitude before its peak;
    with the peak about 30 steps in (f0 = 5.65 at 0.9 dt_crit), the steepest case for
    the check intervals used here, the onset is never taken for an instability."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, _, _ = c1
    s = Solver(cfg, precision="fp64")
    dtc = s.critical_dt()
    u, d = s.zeros(1), s.zeros(1)
    out = fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=[dict(x=(0.1, 0.1), f0=5.65)],
                        dt=0.9 * dtc, nsteps=600, start=1, check_every=check_every)])
    torch.cuda.synchronize()
    assert out[0]["status"] == fcw.FCW_OK and out[0]["steps_done"] == 600
    s.close()


def test_energy_matches_oracle(c1):
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, disc, dt = c1
    nsteps = 180
    s = Solver(cfg, precision="fp64")
    u, d = s.zeros(1), s.zeros(1)
    out = fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=SRC2[:1], dt=dt, nsteps=nsteps,
                        start=1, energy=True)])
    torch.cuda.synchronize()
    r = timestep.cdm(disc, dt, nsteps, sources=SRC2[:1])
    e_ref = timestep.energy(disc, r["u_prev"], r["u"], dt)
    assert e_ref > 0
    assert out[0]["energy"][0] == pytest.approx(e_ref, rel=1e-9)
    s.close()


def test_receiver_errors_and_boundary_points(c1):
    """A receiver outside the box is refused; one on the hole's surface or inside the hole
    reads the fictitious-domain field there, as the oracle's observer rows do."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, disc, dt = c1
    s = Solver(cfg, precision="fp64")
    u, d = s.zeros(1), s.zeros(1)
    tr = _traces_buf(1, 5, 1)
    with pytest.raises(fcw.FcwError) as e:
        fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, dt=dt, nsteps=5, start=1,
                      receivers=[(1.2, 0.3)], traces=tr)])
    assert e.value.status == fcw.FCW_E_ARG
    rec = [(0.75, 0.5), (0.6, 0.55)]  # on the hole's surface; inside the hole
    nsteps = 120
    tr = _traces_buf(1, nsteps, len(rec))
    fcw.run([dict(ctx=s.ctx, nrhs=1, u=u, d=d, sources=SRC2[:1], dt=dt, nsteps=nsteps, start=1,
                  receivers=rec, traces=tr)])
    torch.cuda.synchronize()
    ref = _oracle_traces(disc, dt, nsteps, SRC2[:1], rec)[0]
    got = tr.cpu().numpy()[0, :, :, 0]
    assert np.abs(ref).max() > 0
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    s.close()


def test_gaussian_source_2d_chunked_and_batched(c1):
    """A volumetric Gaussian source (and a point source on the second right-hand side):
    fcw_step_explicit in two calls against the oracle (FP64, 1e-10); fcw_run with a second
    problem in the same launches equals the problem run alone in one call, bit for bit,
    and the second problem matches its oracle run."""
    import torch
    from paper_2501_19013_amd import fcw
    from paper_2501_19013_amd.solver import Solver
    cfg, disc, dt = c1
    srcs = [dict(x=(0.2, 0.15), sigma=0.03, f0=10.0, amp=1.0), SRC2[1]]
    nsteps = 130
    refs = [timestep.cdm(disc, dt, nsteps, sources=[q])["u"] for q in srcs]
    s = Solver(cfg, precision="fp64")
    u, d = s.zeros(2), s.zeros(2)
    s.step(u, d, srcs, dt, 47, start=True)
    s.step(u, d, srcs, dt, nsteps - 47, t0=47 * dt)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for q in range(2):
        assert np.linalg.norm(got[q] - refs[q]) <= 1e-10 * np.linalg.norm(refs[q]), q
    # batched with another problem of the same kind
    cfg2 = dict(cfg)
    cc, rr = workloads.random_circles(seed=43, count=5, rmin=0.03, rmax=0.07,
                                      keep_clear=((0.1, 0.1), (0.7, 0.3), (0.2, 0.15)))
    cfg2.update(ncells=(20, 20), void_center=cc, void_radius=rr)
    s2 = Solver(cfg2, precision="fp64")
    dt2 = 0.9 * s2.critical_dt()
    ua, da = s.zeros(2), s.zeros(2)
    ub, db = s2.zeros(2), s2.zeros(2)
    fcw.run([dict(ctx=s.ctx, nrhs=2, u=ua, d=da, sources=srcs, dt=dt, nsteps=nsteps, start=1),
             dict(ctx=s2.ctx, nrhs=2, u=ub, d=db, sources=srcs, dt=dt2, nsteps=90, start=1)])
    # the same problem alone in one call (one call: the same source times as the batch)
    u1, d1 = s.zeros(2), s.zeros(2)
    s.step(u1, d1, srcs, dt, nsteps, start=True)
    torch.cuda.synchronize()
    assert np.array_equal(ua.cpu().numpy(), u1.cpu().numpy())
    disc2 = problem.build(problem.Problem.from_config(cfg2))
    ref2 = timestep.cdm(disc2, dt2, 90, sources=[srcs[0]])["u"]
    assert np.linalg.norm(ub[0].cpu().numpy() - ref2) <= 1e-10 * np.linalg.norm(ref2)
    s.close()
    s2.close()
