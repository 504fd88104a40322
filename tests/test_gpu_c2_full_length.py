"""The benchmarked 2-D workload at its full length against the oracle.

512 x 512 cells, p = 4, 40 random circular voids (seed 2), Ricker f0 = 10 at (0.1, 0.1),
dt = 0.9 dt_crit with dt_crit = 2 / sqrt(lambda_max) from the oracle's own eigen-solve:
the device steps 2000 times in FP32 (the benchmarked form, autotuned kernel) and in FP64;
after steps 500, 1000, 1500 and 2000 the relative L2 error over all DOFs against the oracle
must stay below 1e-4 (FP32) and 1e-10 (FP64).

The tests run in file order and share state: each one advances the oracle and both device
runs from the previous checkpoint, so no single test runs long."""
import numpy as np
import pytest

import workloads
from oracle import problem, timestep

pytestmark = pytest.mark.gpu

CHECKPOINTS = (500, 1000, 1500, 2000)
TOL = {"fp32": 1e-4, "fp64": 1e-10}
_state = {}


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_c2_setup():
    from paper_2501_19013_amd.solver import Solver
    cfg = workloads.config("c2")
    disc = problem.build(problem.Problem.from_config(cfg))
    dt = 0.9 * timestep.critical_dt(disc, tol=1e-10)
    runs = {}
    for precision in ("fp32", "fp64"):
        s = Solver(cfg, precision=precision)
        if precision == "fp32":
            s.autotune(1, 20)
        runs[precision] = (s, s.zeros(1), s.zeros(1))
    _state.update(cfg=cfg, disc=disc, dt=dt, runs=runs, k=0, orc=None)
    assert 1e-6 < dt < 1e-3
    print(f"c2 full length: dt = {dt:.6e}, {len(disc.cut_cells)} cut cells", flush=True)


@pytest.mark.parametrize("k", CHECKPOINTS)
def test_c2_full_length(k):
    import torch
    if not _state:
        pytest.skip("set-up test did not run")
    cfg, disc, dt = _state["cfg"], _state["disc"], _state["dt"]
    src = cfg["sources"]
    k0 = _state["k"]
    assert k > k0
    orc = timestep.cdm(disc, dt, k, sources=src, resume=_state["orc"])
    _state["orc"] = orc
    errs = {}
    for precision, (s, u, d) in _state["runs"].items():
        s.step(u, d, src, dt, k - k0, t0=k0 * dt, start=(k0 == 0))
        torch.cuda.synchronize()
        errs[precision] = rel_l2(u[0].double().cpu().numpy(), orc["u"])
    _state["k"] = k
    print(f"c2 step {k}: rel L2 vs oracle fp32 {errs['fp32']:.3e} fp64 {errs['fp64']:.3e}",
          flush=True)
    assert np.linalg.norm(orc["u"]) > 0
    for precision, e in errs.items():
        assert e <= TOL[precision], (precision, k, e)
