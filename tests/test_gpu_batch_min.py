"""Batched sigma_min run (Algorithm 2 for many matrices x 8 starts) and
batched kappa, against the plain run and the oracle.

Every matrix is factored by the same host LU as the single-matrix plan, so
each (matrix, start) pair runs the plain method's arithmetic: only the
order of additions inside the solves' sums (8 sides per pass) and the
global sums differs. So each pair's ||A^-1 x|| must follow the plain run
from the same start to rounding and stop at the same update as the oracle,
and each matrix's kappa must match the oracle's to 1e-3.
"""

import json
import os

import numpy as np
import pytest

from oracle import PAOptions, estimate_cond as oracle_estimate
from oracle.inverse import LUInverse
from oracle.padam import projected_adam
from stoprule import assert_same_stop
from synth import hm_batch_specs, hydromech2d, start_block, start_vector

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2409_11515_amd as pa

    pa._binding.lib()
    return torch


def _mats(sides, seed=5):
    specs = hm_batch_specs(count=len(sides), side_range=(min(sides), max(sides)), seed_sides=seed,
                           seed_base=seed + 1)
    return [hydromech2d(s, log_eta=specs[i][1][:s - 1, :s - 1], log_k=specs[i][2][:s - 1, :s - 1])
            for i, s in enumerate(sides)]


def test_batch_min_matches_plain_runs(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    mats = [hydromech2d(s, seed=20 + s) for s in (6, 11, 9, 15)]
    starts = [start_block(m.n, 8, 300 + i) for i, m in enumerate(mats)]
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in mats], sigma_min=True).bind()
    r = b.run_min(torch.as_tensor(pa.interleave_starts(starts), device="cuda"), max_iter=300,
                  trace=True)
    b.close()
    assert np.all(r["pair_iters"] == 300)
    for i, m in enumerate(mats):
        p = pa.Plan(m.n, m.rowptr, m.col, m.val).bind()
        for k in range(8):
            g = p.run(None, torch.as_tensor(starts[i][k], device="cuda"), max_iter=300, trace=True)
            assert r["pair_best"][i, k] == pytest.approx(1.0 / g["sigma_min"], rel=1e-10)
            np.testing.assert_allclose(r["trace"][i, k, :50], g["trace_min"][:50], rtol=1e-10)
        p.close()
        assert r["sigma_min"][i] == 1.0 / r["pair_best"][i].max()


def test_batch_min_stop_rule_matches_oracle(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    mats = [hydromech2d(s, seed=40 + s) for s in (12, 7, 19)]
    starts = [start_block(m.n, 8, 500 + i) for i, m in enumerate(mats)]
    opts = dict(max_iter=4000, stop_rtol=1e-9, stop_window=50, alpha_min=1.25e-3, alpha_decay=0.5)
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in mats], sigma_min=True).bind()
    r = b.run_min(torch.as_tensor(pa.interleave_starts(starts), device="cuda"), **opts)
    b.close()
    for i, m in enumerate(mats):
        inv = LUInverse(m.n, m.rowptr, m.col, m.val)
        for k in (0, 6):
            o = projected_adam(inv.apply, inv.evaluate, starts[i][k], PAOptions(**opts))
            # the oracle solves with SuperLU's factors, the batch with the
            # library's: over thousands of updates the bests drift apart at
            # the 1e-7 level (the plain path's floor test holds 1e-6 too)
            assert_same_stop(r["pair_iters"][i, k], r["pair_best"][i, k], o, opts["stop_rtol"],
                             opts["stop_window"], 1e-6, (i, k))


def test_batched_kappa_matches_oracle_with_a_201_system(torch_cuda):
    """estimate_batched over uneven systems, one of them the 201x201-node
    system of the stored golden run: the pair that starts from the golden's
    start vectors reproduces its kappa, and every matrix's kappa (best over
    its 8 starts) matches the oracle's to 1e-3."""
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    with open(os.path.join(GOLDEN, "hm_side201_seed1.json")) as f:
        gold = json.load(f)
    big = hydromech2d(201, seed=1)
    small = [hydromech2d(s, seed=60 + s) for s in (8, 14, 23)]
    mats = small + [big]
    o = gold["opts"]
    opts = dict(alpha=o["alpha"], alpha_min=o["alpha_min"], alpha_decay=o["alpha_decay"],
                beta1=o["beta1"], beta2=o["beta2"], eps=o["eps"], stop_rtol=o["stop_rtol"],
                stop_window=o["stop_window"], max_iter=o["max_iter"])
    smax = [start_block(m.n, 8, 700 + i) for i, m in enumerate(mats)]
    smin = [start_block(m.n, 8, 800 + i) for i, m in enumerate(mats)]
    smax[-1][0] = start_vector(big.n, 11)  # the golden run's starts
    smin[-1][0] = start_vector(big.n, 12)
    res = pa.estimate_batched([(m.n, m.rowptr, m.col, m.val) for m in mats],
                              torch.as_tensor(pa.interleave_starts(smax), device="cuda"),
                              torch.as_tensor(pa.interleave_starts(smin), device="cuda"), **opts)
    assert abs(res[-1]["kappa"] / gold["kappa"] - 1.0) <= 1e-3
    for i, m in enumerate(small):
        # the oracle from the best of the batch's own starts: every start is
        # run; kappa = best sigma_max / best sigma_min
        best_max = max(oracle_estimate(m.n, m.rowptr, m.col, m.val, smax[i][k],
                                       opts=PAOptions(**opts), min_method="lu")["sigma_max"]
                       for k in range(8))
        inv = LUInverse(m.n, m.rowptr, m.col, m.val)
        best_inv = max(projected_adam(inv.apply, inv.evaluate, smin[i][k], PAOptions(**opts)).sigma
                       for k in range(8))
        assert res[i]["kappa"] == pytest.approx(best_max * best_inv, rel=1e-3), i
        assert res[i]["status_max"] == 0 and res[i]["status_min"] == 0


def test_running_matrix_unaffected_by_stopped_ones(torch_cuda):
    """Once a matrix's starts have all stopped, the solves walk only the
    running matrices' tasks (the lists cut down on the device) and the
    element kernels skip its tiles. None of this may touch a running
    matrix's arithmetic: with the same row tiles, each matrix's run in a
    batch whose other matrices stop at other updates is bit for bit its run
    alone."""
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    mats = [hydromech2d(17, seed=91)] + [hydromech2d(s, seed=92 + s) for s in (5, 7)]
    opts = dict(max_iter=3000, stop_rtol=1e-6, stop_window=25)
    starts = [start_block(m.n, 8, 910 + i) for i, m in enumerate(mats)]

    def run(ms, ss):
        b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in ms], sigma_min=True).bind(tile_rows=64,
                                                                                       grid=1024)
        r = b.run_min(torch.as_tensor(pa.interleave_starts(ss), device="cuda"), trace=True, **opts)
        b.close()
        return r

    r = run(mats, starts)
    last = r["pair_iters"].max(axis=1)
    # the matrices stop at different updates: the later ones ran on with
    # the earlier ones' tasks cut from the lists
    assert last.min() < last.max()
    for i, m in enumerate(mats):
        r1 = run([m], [starts[i]])
        np.testing.assert_array_equal(r["pair_iters"][i], r1["pair_iters"][0])
        np.testing.assert_array_equal(r["pair_best"][i], r1["pair_best"][0])
        np.testing.assert_array_equal(r["trace"][i], r1["trace"][0])
