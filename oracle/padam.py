"""Algorithm 1 (Projected Adam), plain float64, one step at a time.

The loss is L(v) = log||v|| - log||M v|| and its gradient (equation
``nabla_loss``) is v/||v||^2 - M^T M v/||M v||^2. Minimising L maximises
||M v||/||v||, so the best value over the iterates is a lower estimate of
||M||_2 (section "Loss Function and Optimization").

Readings where the paper is silent (each listed in the design notes):

* x_init is normalised before the loop (the tangent projection assumes a
  unit vector);
* the loss is tracked as sigma = sqrt(||M x||^2 / ||x||^2), which orders the
  iterates exactly as L does; the candidates are x_1 .. x_T (x_init is never
  evaluated: L_min starts at infinity and the check follows the update), the
  evaluation of x_t reuses the product M x_t that the next gradient needs,
  and x_T costs one extra product; a strict ">" keeps the earliest best;
* the bias corrections use running products beta^t = beta^(t-1) * beta;
* x . x is computed as a dot product, not assumed to be 1;
* optional early stop (off by default): after T updates, T a multiple of the
  window W with T >= 2W, stop when best_T - best_(T-W) <= rtol * best_T.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class PAOptions:
    alpha: float = 1.0e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1.0e-8
    max_iter: int = 20000
    stop_rtol: float = 0.0
    stop_window: int = 0
    # Step-size floor (not in the paper; 0 = Algorithm 1 as written). When the
    # stop rule fires and alpha > alpha_min, the run continues with
    # alpha = max(alpha * alpha_decay, alpha_min), moments kept, and stops at
    # the first plateau reached at the floor.
    alpha_min: float = 0.0
    alpha_decay: float = 0.5


@dataclass
class PAResult:
    sigma: float  # best ||M x|| / ||x|| over the evaluated iterates
    x_best: np.ndarray  # the iterate that attained it
    iters: int  # number of Adam updates performed (T)
    trace: np.ndarray = field(repr=False)  # trace[t-1] = best over x_1 .. x_t
    stopped_early: bool = False


def _stop_now(trace, T, opts: PAOptions) -> bool:
    w = opts.stop_window
    if w <= 0 or opts.stop_rtol <= 0.0 or T % w != 0 or T < 2 * w:
        return False
    return trace[T - 1] - trace[T - 1 - w] <= opts.stop_rtol * trace[T - 1]


def projected_adam(apply, evaluate, x0, opts: PAOptions, observer=None) -> PAResult:
    """Run Algorithm 1.

    ``apply(x)`` returns (M x, M^T M x); ``evaluate(x)`` returns M x.
    ``observer(t, x_prev, g, d, x_next)``, if given, sees every update (tests).
    """
    x = np.array(x0, dtype=np.float64)
    nrm0 = np.sqrt(x @ x)
    if not np.isfinite(nrm0) or nrm0 == 0.0:
        raise ValueError("start vector must be finite and non-zero")
    x = x / nrm0
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    b1, b2 = opts.beta1, opts.beta2
    b1t = 1.0
    b2t = 1.0
    best = -np.inf
    x_best = x.copy()
    trace = []
    alpha = opts.alpha

    def consider(xc, y):
        nonlocal best, x_best
        sigma = np.sqrt((y @ y) / (xc @ xc))
        if sigma > best:
            best = sigma
            x_best = xc.copy()
        trace.append(best)

    for t in range(1, opts.max_iter + 1):
        y, w = apply(x)  # y = M x_(t-1), w = M^T M x_(t-1)
        if t >= 2:
            consider(x, y)  # evaluation of x_(t-1)
            if _stop_now(trace, t - 1, opts):
                if opts.alpha_min > 0.0 and alpha > opts.alpha_min:
                    alpha = max(alpha * opts.alpha_decay, opts.alpha_min)
                else:
                    return PAResult(best, x_best, t - 1, np.asarray(trace), True)
        nx2 = x @ x
        ny2 = y @ y
        g = x / nx2 - w / ny2  # equation nabla_loss
        m = b1 * m + (1.0 - b1) * g  # biased first moment
        v = b2 * v + (1.0 - b2) * (g * g)  # biased second moment
        b1t = b1t * b1
        b2t = b2t * b2
        m_hat = m / (1.0 - b1t)
        v_hat = v / (1.0 - b2t)
        d = alpha * m_hat / (np.sqrt(v_hat) + opts.eps)
        d = d - (x @ d) * x  # tangent to the unit sphere
        x_prev = x
        x = x - d
        x = x / np.sqrt(x @ x)  # back onto the unit sphere
        if observer is not None:
            observer(t, x_prev, g, d, x)
    if opts.max_iter >= 1:
        consider(x, evaluate(x))  # evaluation of x_T
    T = opts.max_iter
    return PAResult(best, x_best, T, np.asarray(trace), False)
