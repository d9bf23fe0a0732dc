"""Update counts of a run against the oracle's, where the stop rule allows it.

The stop rule (and the step-size floor's halving) decides at every window
boundary T by comparing the window's gain, best(T) - best(T - w), with
stop_rtol * best(T). Two runs that differ only in the rounding of their
global sums follow trajectories that drift apart at the rounding level, and
a boundary whose gain lies close to the threshold can then be decided either
way. Such a boundary is found from the oracle's own trace alone: its gain
lies within a factor of two of the threshold. When every boundary the oracle
decided is clear of that band, the update counts must be equal; otherwise
they may differ by the stop windows the close boundaries can shift, and the
best values must still agree.
"""

import numpy as np


def close_boundaries(trace, iters, stop_rtol, stop_window, band=2.0):
    """Window boundaries T <= iters (T >= 2 w) of the oracle's run whose gain
    lies within [threshold / band, threshold * band]."""
    tr = np.asarray(trace)
    out = []
    w = stop_window
    if w <= 0 or stop_rtol <= 0:
        return out
    for T in range(2 * w, iters + 1, w):
        gain = tr[T - 1] - tr[T - 1 - w]
        thr = stop_rtol * tr[T - 1]
        if thr / band <= gain <= thr * band:
            out.append(T)
    return out


def assert_same_stop(iters, sigma, o, stop_rtol, stop_window, rel, what=""):
    """iters, sigma: the run under test; o: the oracle's PAResult."""
    close = close_boundaries(o.trace, o.iters, stop_rtol, stop_window)
    if not close:
        assert iters == o.iters, (what, iters, o.iters)
    else:
        assert abs(int(iters) - int(o.iters)) <= stop_window * len(close), (what, iters, o.iters, close)
    assert abs(sigma - o.sigma) <= rel * abs(o.sigma), (what, sigma, o.sigma)
