"""GPU tests of the serving loop: requests of different geometries, dimensions, degrees,
sizes and step counts arrive over time, are admitted as slots and memory free up and are
advanced together in quanta.  Each served result must equal the same request served
alone bit for bit (the same kernels and quantum boundaries run on it; only the company
differs), and a served FP32 result must stay within 1e-4 relative L2 of the FP64 oracle."""
import copy

import numpy as np
import pytest

import workloads
from oracle import problem, timestep

pytestmark = pytest.mark.gpu

# (dim, cells per side, p, void seed, steps, arrival in s)
# (step counts are large enough that a request stays resident for many quanta while
# later ones are set up and join)
SPECS = [(2, 24, 4, 31, 1500, 0.0), (2, 17, 3, 32, 900, 0.0), (3, 5, 2, 33, 600, 0.01),
         (2, 30, 4, 34, 1200, 0.02), (3, 4, 3, 35, 500, 0.03), (2, 21, 2, 36, 800, 0.04),
         (2, 13, 4, 37, 700, 0.05), (3, 6, 2, 38, 400, 0.06)]


def _requests():
    from paper_2501_19013_amd.serve import Request
    out = []
    for i, (dim, n, p, seed, steps, t) in enumerate(SPECS):
        cfg = workloads.scaled_config(dim, n, p, seed, nsteps=steps,
                                      depth=3 if dim == 2 else 2)
        out.append(Request(rid=i, cfg=cfg, nsteps=steps, arrival=t, sources=cfg["sources"]))
    return out


@pytest.fixture(scope="module")
def served():
    from paper_2501_19013_amd.serve import Server, estimate_footprint
    reqs = _requests()
    # room for about three of the larger problems at once: later ones wait for memory
    budget = 3 * max(estimate_footprint(r.cfg, 1, "fp32") for r in reqs)
    srv = Server(precision="fp32", max_slots=4, quantum=16, keep_results=True,
                 memory_budget=budget)
    metrics = srv.run(reqs)
    yield srv, reqs, metrics, budget
    srv.close()


def test_every_request_served(served):
    _, reqs, m, budget = served
    assert m["n"] == len(reqs)
    assert all(r.done is not None and r.done >= r.arrival for r in reqs)
    assert 0 < m["p50_latency_s"] <= m["p99_latency_s"]
    assert m["dof_updates_per_s"] > 0
    # requests overlapped on the device, and admission kept within the memory budget
    assert m["max_resident"] >= 2
    assert m["peak_reserved_bytes"] <= budget
    for r in reqs:
        assert np.all(np.isfinite(r.state)) and np.abs(r.state).max() > 0


def test_mix_equals_alone(served):
    srv, reqs, _, _ = served
    for r in reqs:
        alone = copy.copy(r)
        alone.arrival, alone.done, alone.state = 0.0, None, None
        srv.run([alone])
        assert alone.dt == r.dt
        assert np.array_equal(alone.state, r.state), f"request {r.rid}"


def test_served_matches_oracle(served):
    _, reqs, _, _ = served
    for r in (reqs[0], reqs[2]):   # one 2-D and one 3-D request
        disc = problem.build(problem.Problem.from_config(r.cfg))
        ref = timestep.cdm(disc, r.dt, r.nsteps, sources=r.sources)["u"]
        got = r.state[0].astype(np.float64)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4, f"request {r.rid}"
