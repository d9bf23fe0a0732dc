"""Pins of the step-size floor (PAOptions.alpha_min), an extension of Algorithm 1.

Until the first plateau the run is Algorithm 1 unchanged, so its trace must
equal the constant-step run's bit for bit; after it, smaller steps can only
raise the running best; and against the exact largest singular value (LAPACK
SVD) the floored run must land much closer than the constant-step run,
whose distance from the optimum the fixed step sets.
"""

import numpy as np

from oracle.padam import PAOptions, projected_adam


def _problem():
    rng = np.random.default_rng(5)
    n = 400
    a = np.diag(np.exp(rng.uniform(0.0, 3.0, n))) + 0.05 * rng.standard_normal((n, n))
    sigma = np.linalg.svd(a, compute_uv=False)[0]
    apply = lambda x: (lambda y: (y, a.T @ y))(a @ x)  # noqa: E731
    return apply, (lambda x: a @ x), rng.standard_normal(n), sigma


def test_floor_is_algorithm_1_until_the_first_plateau_then_closer_to_the_svd():
    apply, ev, x0, sigma = _problem()
    plain = projected_adam(apply, ev, x0, PAOptions(max_iter=3000, stop_rtol=1e-8, stop_window=50))
    floor = projected_adam(apply, ev, x0, PAOptions(max_iter=6000, stop_rtol=1e-8, stop_window=50,
                                                    alpha_min=1e-4))
    assert plain.stopped_early and floor.stopped_early
    t1 = plain.iters
    np.testing.assert_array_equal(floor.trace[:t1], plain.trace[:t1])
    assert floor.iters > t1 and floor.sigma >= plain.sigma
    err_plain = (sigma - plain.sigma) / sigma
    err_floor = (sigma - floor.sigma) / sigma
    assert 0.0 <= err_floor < 0.1 * err_plain, (err_plain, err_floor)
    assert err_floor < 1e-7


def test_floor_zero_or_equal_to_alpha_is_the_plain_run():
    apply, ev, x0, _ = _problem()
    base = PAOptions(max_iter=800, stop_rtol=1e-8, stop_window=50)
    plain = projected_adam(apply, ev, x0, base)
    same = projected_adam(apply, ev, x0, PAOptions(max_iter=800, stop_rtol=1e-8, stop_window=50,
                                                   alpha_min=base.alpha))
    assert same.iters == plain.iters and same.sigma == plain.sigma
