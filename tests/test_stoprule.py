"""The close-boundary rule of tests/stoprule.py on synthetic traces and on
the oracle run whose decision at one window boundary sits near the stop
threshold (the step-size-floor batch case of tests/test_gpu_batch.py)."""

import numpy as np

from oracle import PAOptions
from oracle.estimate import forward_apply
from oracle.padam import projected_adam
from stoprule import assert_same_stop, close_boundaries
from synth import hydromech2d, start_block


def test_close_boundaries_synthetic():
    # best values with window gains 1e-3, 1.5e-9, 1e-12 (relative) at T = 20, 30, 40
    tr = np.ones(40)
    tr[10:20] += 1e-3
    tr[20:30] = tr[19] * (1 + 1.5e-9)
    tr[30:40] = tr[29] * (1 + 1e-12)
    assert close_boundaries(tr, 40, 1e-9, 10) == [30]
    assert close_boundaries(tr, 40, 1e-3, 10) == [20]
    assert close_boundaries(tr, 40, 0.0, 10) == []


class _R:
    def __init__(self, iters, sigma, trace):
        self.iters, self.sigma, self.trace = iters, sigma, trace


def test_assert_same_stop():
    tr = np.linspace(1.0, 2.0, 100)
    o = _R(100, 2.0, tr)
    assert_same_stop(100, 2.0, o, 1e-9, 10, 1e-12)  # no close boundary: equal counts
    try:
        assert_same_stop(90, 2.0, o, 1e-9, 10, 1e-12)
        raise RuntimeError("a differing count passed")
    except AssertionError:
        pass


def test_floor_case_has_a_close_boundary():
    m = hydromech2d(6, seed=4)
    x0 = start_block(m.n, 8, 1001)[1]
    opts = dict(max_iter=6000, stop_rtol=1e-9, stop_window=50, alpha_min=1.25e-3, alpha_decay=0.5)
    apply, evaluate = forward_apply(m.n, m.rowptr, m.col, m.val)
    o = projected_adam(apply, evaluate, x0, PAOptions(**opts))
    assert o.iters == 1750
    assert close_boundaries(o.trace, o.iters, 1e-9, 50) == [1600]
