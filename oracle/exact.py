"""Exact references that pin the oracle, independent of Projected Adam.

* closed forms: singular values of diagonal and 2x2 block-diagonal matrices;
* brute force for tiny dense matrices in extended precision (mpmath):
  - ``sv_extremes_mp_svd``: the full singular value decomposition at ``dps``
    digits (the definition of kappa_2 through singular values);
  - ``sv_extremes_mp_inverse``: A^-1 computed exactly enough at ``dps``
    digits, rounded to float64, then sigma_max(A) and sigma_max(A^-1) from
    LAPACK's SVD. The largest singular value is perturbed only by about
    eps*sqrt(n) relative under the final rounding, so this gives both
    extremes to ~1e-14 even at kappa ~ 1e24, where a float64 SVD of A alone
    is wrong in sigma_min by orders of magnitude.
"""

from __future__ import annotations

import math

import numpy as np


def sv_2x2(a, b, c, d):
    """(sigma_1, sigma_2) of [[a, b], [c, d]], computed stably.

    With F = ||B||_F^2 and det = ad - bc: sigma_1^2 = (F + sqrt(F^2 - 4 det^2))/2
    and sigma_2 = |det| / sigma_1, where F^2 - 4 det^2 is formed as the product
    ((a-d)^2 + (b+c)^2) ((a+d)^2 + (b-c)^2) to avoid cancellation.
    """
    f = a * a + b * b + c * c + d * d
    det = a * d - b * c
    disc = math.sqrt(((a - d) ** 2 + (b + c) ** 2) * ((a + d) ** 2 + (b - c) ** 2))
    s1 = math.sqrt((f + disc) / 2.0)
    s2 = abs(det) / s1 if s1 > 0 else 0.0
    return s1, s2


def kappa_blockdiag2(blocks):
    """kappa_2 of a block-diagonal matrix of 2x2 blocks: max sigma_1 / min sigma_2."""
    svs = [sv_2x2(*np.asarray(b, dtype=np.float64).ravel()) for b in blocks]
    smax = max(s[0] for s in svs)
    smin = min(s[1] for s in svs)
    return smax, smin, smax / smin


def sv_extremes_mp_svd(dense, dps: int = 50):
    """(sigma_max, sigma_min) from mpmath's SVD at ``dps`` decimal digits."""
    import mpmath as mp

    with mp.workdps(dps):
        s = mp.svd_r(mp.matrix(np.asarray(dense, dtype=np.float64).tolist()), compute_uv=False)
        vals = [float(v) for v in s]
    return max(vals), min(vals)


def sv_extremes_mp_inverse(dense, dps: int = 40):
    """(sigma_max, sigma_min) via an extended-precision inverse (see module doc)."""
    import mpmath as mp

    a = np.asarray(dense, dtype=np.float64)
    with mp.workdps(dps):
        inv = mp.inverse(mp.matrix(a.tolist()))
        inv64 = np.array([[float(inv[i, j]) for j in range(a.shape[1])] for i in range(a.shape[0])])
    smax = float(np.linalg.svd(a, compute_uv=False)[0])
    inv_norm = float(np.linalg.svd(inv64, compute_uv=False)[0])
    return smax, 1.0 / inv_norm
