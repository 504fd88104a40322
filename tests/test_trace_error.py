"""The accuracy measure of Sec. 3.2 (eq. error): the library's host function against the
oracle's and against values the definition fixes (no GPU needed)."""
import numpy as np
import pytest

from oracle import metrics


def test_closed_forms():
    ref = np.array([[1.0, 2.0], [3.0, -4.0]])
    assert metrics.trace_error(ref, ref) == 0.0
    # a trace scaled by (1 + a) has relative error |a|; the mean over observers
    sim = ref * np.array([1.1, 0.7])
    assert metrics.trace_error(sim, ref) == pytest.approx(0.5 * (0.1 + 0.3), rel=1e-14)


def test_library_matches_the_oracle_and_samples_rows():
    from paper_2501_19013_amd import fcw
    rng = np.random.default_rng(3)
    ns, nobs = 100, 11
    # the simulation every step (500 steps), the reference every step of half the size
    sim = rng.standard_normal((501, nobs))
    ref = rng.standard_normal((1001, nobs))
    e = fcw.trace_error(sim, ref, 5, 10, ns)
    want = metrics.trace_error(sim[5::5][:ns], ref[10::10][:ns])
    assert e == pytest.approx(want, rel=1e-13)
    assert fcw.trace_error(ref, ref, 10, 10, ns) == 0.0
    with pytest.raises(fcw.FcwError):
        fcw.trace_error(sim, np.zeros_like(ref), 5, 10, ns)
