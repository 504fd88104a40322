"""Accuracy measure of the paper (Sec. 3.2, eq. error): the relative L2 error of the
observer traces over n_s equidistant time samples, averaged over the observers.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np


def trace_error(sim, ref):
    """e = 1/n_p sum_i ||sim[:, i] - ref[:, i]||_2 / ||ref[:, i]||_2 for traces sampled at
    the same n_s times (arrays [n_s][n_p])."""
    sim = np.asarray(sim, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    per = [np.linalg.norm(sim[:, i] - ref[:, i]) / np.linalg.norm(ref[:, i])
           for i in range(ref.shape[1])]
    return float(np.mean(per))
