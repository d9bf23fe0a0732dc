"""Ablation, not the paper's method: sigma_min by minimising ||A x|| / ||x||.

The paper computes ||A^-1||_2 = 1/sigma_min with Algorithm 2 (one LU and
triangular solves). The obvious alternative that needs only products with A
and A^T is to run the same Projected Adam iteration the other way round:
descend on L'(v) = log||A v|| - log||v||, whose gradient is the negative of
equation ``nabla_loss``, A^T A v/||A v||^2 - v/||v||^2, and keep the smallest
||A x|| / ||x|| seen. Every value is an upper bound of sigma_min. At the
condition numbers of the paper's systems it does not converge in any
practical number of updates (the slowest direction of A^T A is the one
sought), which is why the paper takes the LU route.

Everything else is Algorithm 1 unchanged: normalised start, bias-corrected
moments with running beta^t products, tangent projection, renormalisation,
candidates x_1 .. x_T with the evaluation of x_t taken from the product the
next gradient needs; a strict "<" keeps the earliest best. The optional stop
rule and step-size floor mirror ``padam``'s with the sense reversed: after T
updates, T a multiple of W and T >= 2W, a plateau is
best_(T-W) - best_T <= rtol * best_T.

TEST INFRASTRUCTURE ONLY (part of the oracle package).
"""

from __future__ import annotations

import numpy as np

from .padam import PAOptions, PAResult


def _plateau(trace, T, opts: PAOptions) -> bool:
    w = opts.stop_window
    if w <= 0 or opts.stop_rtol <= 0.0 or T % w != 0 or T < 2 * w:
        return False
    return trace[T - 1 - w] - trace[T - 1] <= opts.stop_rtol * trace[T - 1]


def minimise_by_spmv(apply, evaluate, x0, opts: PAOptions) -> PAResult:
    """Smallest ||M x|| / ||x|| reached by Projected Adam descending on L'.

    ``apply(x)`` returns (M x, M^T M x); ``evaluate(x)`` returns M x. The
    returned ``sigma`` is the best (smallest) value, an upper bound of
    sigma_min(M).
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
    best = np.inf
    x_best = x.copy()
    trace = []
    alpha = opts.alpha

    def consider(xc, y):
        nonlocal best, x_best
        sigma = np.sqrt((y @ y) / (xc @ xc))
        if sigma < best:
            best = sigma
            x_best = xc.copy()
        trace.append(best)

    for t in range(1, opts.max_iter + 1):
        y, w = apply(x)
        if t >= 2:
            consider(x, y)
            if _plateau(trace, t - 1, opts):
                if opts.alpha_min > 0.0 and alpha > opts.alpha_min:
                    alpha = max(alpha * opts.alpha_decay, opts.alpha_min)
                else:
                    return PAResult(best, x_best, t - 1, np.asarray(trace), True)
        nx2 = x @ x
        ny2 = y @ y
        g = w / ny2 - x / nx2  # minus equation nabla_loss
        m = b1 * m + (1.0 - b1) * g
        v = b2 * v + (1.0 - b2) * (g * g)
        b1t = b1t * b1
        b2t = b2t * b2
        m_hat = m / (1.0 - b1t)
        v_hat = v / (1.0 - b2t)
        d = alpha * m_hat / (np.sqrt(v_hat) + opts.eps)
        d = d - (x @ d) * x
        x = x - d
        x = x / np.sqrt(x @ x)
    if opts.max_iter >= 1:
        consider(x, evaluate(x))
    return PAResult(best, x_best, opts.max_iter, np.asarray(trace), False)
