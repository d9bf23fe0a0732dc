"""The oracle against stored extended-precision references (tests/golden/).

c1_stokes_10x10_seed0.json: the tiny Stokes system's extreme singular values
from mpmath's SVD at 50 digits (and, agreeing to 1e-15, from an mpmath
inverse). hm_side6_seed1.json: a small six-field hydro-mechanical system,
mpmath inverse. Both files are written by tests/golden/make_golden.py, which
calls only the oracle's exact references and the generators.
"""

import json
import os

import numpy as np
import pytest

from oracle import PAOptions, estimate_cond
from synth import hydromech2d, start_vector, stokes2d

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_c1_stokes_matches_dense_svd():
    g = _load("c1_stokes_10x10_seed0.json")
    a = stokes2d(10, 10, seed=0)
    assert (a.n, a.nnz) == (g["n"], g["nnz"])
    r = estimate_cond(a.n, a.rowptr, a.col, a.val, start_vector(a.n, 1),
                      opts=PAOptions(max_iter=20000))
    assert r["kappa"] == pytest.approx(g["kappa_svd"], rel=1e-6)
    assert r["sigma_max"] == pytest.approx(g["sigma_max_svd"], rel=1e-6)
    assert r["sigma_min"] == pytest.approx(g["sigma_min_svd"], rel=1e-6)
    # one-sided: estimates never exceed the truth (up to rounding)
    assert r["sigma_max"] <= g["sigma_max_svd"] * (1 + 1e-12)
    assert r["sigma_min"] >= g["sigma_min_svd"] * (1 - 1e-12)


def test_hm_small_matches_extended_precision():
    g = _load("hm_side6_seed1.json")
    a = hydromech2d(6, seed=1)
    assert (a.n, a.nnz) == (g["n"], g["nnz"])
    r = estimate_cond(a.n, a.rowptr, a.col, a.val, start_vector(a.n, 2),
                      opts=PAOptions(max_iter=5000))
    assert r["kappa"] == pytest.approx(g["kappa_inv"], rel=1e-6)


def test_generator_statistics_match_paper_shape():
    # column norms in two clusters (< 1e-2 and > 1e10), one third small, as
    # the paper's column-norm distribution; kappa far above 1/eps
    a = hydromech2d(16, seed=1)
    d = a.to_scipy().toarray()
    cn = np.sqrt((d * d).sum(0))
    assert np.mean(cn < 1e-2) == pytest.approx(1 / 3, abs=1e-12)
    assert np.mean(cn > 1e10) == pytest.approx(2 / 3, abs=1e-12)
    assert a.n == 6 * 16 * 16
