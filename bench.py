"""Benchmark: time-to-kappa of the Projected Adam estimator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload hm201|hm1001|stokes10|c4batch|c5warm]

One step = one full estimate of kappa_2 for one matrix: the sigma_max run
(SpMV with A and A^T, global norms, fused Adam moment update and projection)
and the sigma_min run (Algorithm 2: four sparse triangular solves per
update), each until the stop rule fires. The matrix, its transpose and the
LU factors are resident in HBM before the timed region (host set-up is
reported apart as setup_s). Prints one JSON line.

Roofline: a profiled run (HIP event pair around every launch, on the plan's
stream) gives each kernel's average duration; the dominant kernel's
algorithmic bytes per launch / duration is "achieved". The SpMV figures are
reported beside it.

cpu_baseline: the CPU oracle (float64, one thread) timed on a bounded sample
of the same workload and scaled to the same iteration counts.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("OMP_NUM_THREADS", "1")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # alpha: initial Adam step, halved on each stop-rule plateau down to the
    # floor (--alpha-min); single systems start large, the batch at 1e-2 since
    # its slowest start sets its time and each halving costs a plateau
    "hm201": dict(kind="hm", side=201, seed=1, golden="hm_side201_seed1.json", min_route=True,
                  alpha=4e-2),
    # 6M rows: the sigma_max run (SpMV / A^T-SpMV / Adam) is the HBM roofline
    # measurement; the host LU of this system is not attempted
    "hm1001": dict(kind="hm", side=1001, seed=2, golden=None, min_route=False, alpha=4e-2),
    "stokes10": dict(kind="stokes", side=10, seed=0, golden="c1_stokes_10x10_seed0.json",
                     min_route=True, alpha=1e-2),
    # 64 matrices, sides U{51..401}, perturbed copies of one base field, 8 starts each
    "c4batch": dict(kind="batch", count=64, side_range=(51, 401), min_route=False, alpha=1e-2),
    # learned warm start: trained on small grids, tested on held-out 201x201 systems
    "c5warm": dict(kind="warm", train=((51, 300), (101, 150)), test_side=201, min_route=True,
                   alpha=4e-2),
}


def bench_warm(w, args):
    """Warm-started vs plain sigma_min runs on held-out systems.

    Training: plain sigma_min runs label the maximisers of ||A^-1 x||/||x|| on
    seeded training matrices of the sides in w["train"] (seeds 10000+), and
    the network is fitted on the device. Test: held-out seeds 20000+ at
    w["test_side"]; per matrix one sigma_max run, the plain (random-start)
    sigma_min run, and the warm-started run with its random-start check and
    fallback; every run stops by the same rule."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import paper_2409_11515_amd as pa
    from paper_2409_11515_amd.warmstart import WarmStart, label
    from synth import hm_fields, hydromech2d, start_vector

    opts = dict(max_iter=args.max_iter, stop_rtol=args.stop_rtol, stop_window=args.stop_window,
                alpha=args.alpha, alpha_min=args.alpha_min, alpha_decay=0.5)
    lab_opts = dict(max_iter=4000, stop_rtol=1e-7, stop_window=50)
    t0 = time.perf_counter()

    def build(seed, side):
        le, lk = hm_fields(side, seed)
        a = hydromech2d(side, log_eta=le, log_k=lk)
        return a, np.stack([le, lk]), pa.Plan(a.n, a.rowptr, a.col, a.val)

    sets = []
    seed0 = 10000
    train = [] if args.params_in else w["train"]
    for side, count in train:
        count = max(16, int(round(count * args.train_scale)))
        fields, labels = [], []
        with ThreadPoolExecutor(max_workers=8) as ex:
            for i, (a, f, plan) in enumerate(ex.map(lambda s: build(s, side),
                                                    range(seed0, seed0 + count))):
                plan.bind()
                u, _ = label(plan, torch.as_tensor(start_vector(a.n, seed0 + i), device="cuda"),
                             **lab_opts)
                plan.close()
                fields.append(f)
                labels.append(u)
                if (i + 1) % 50 == 0:
                    print(f"[bench] labelled {i + 1}/{count} at side {side} "
                          f"({time.perf_counter() - t0:.0f}s)", file=sys.stderr, flush=True)
        seed0 += count
        sets.append((torch.as_tensor(np.asarray(fields), device="cuda").contiguous(),
                     torch.stack(labels).contiguous()))
    label_s = time.perf_counter() - t0
    ws = WarmStart(16, max(w["test_side"], max(s for s, _ in w["train"])), seed=0,
                   params=np.load(args.params_in) if args.params_in else None)
    t0 = time.perf_counter()
    hist = [float("nan")]
    if sets:
        hist = ws.fit_sets(sets, epochs=args.epochs, batch=16, lr=2e-3, lr_final=1e-4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    if args.params_out:
        np.save(args.params_out, ws.params())
    print(f"[bench] trained {args.epochs if sets else 0} epochs in {train_s:.1f}s, loss "
          f"{hist[0]:.3f} -> {hist[-1]:.3f}", file=sys.stderr, flush=True)

    side = w["test_side"]
    rows = []
    fwd_ms = []
    with ThreadPoolExecutor(max_workers=min(8, args.test_count)) as ex:
        first = 20000 + args.test_first
        futs = [ex.submit(build, s, side) for s in range(first, first + args.test_count)]
        for i, fu in enumerate(futs):
            a, f, plan = fu.result()
            plan.bind()
            seed = first + i
            xr = torch.as_tensor(start_vector(a.n, seed + 7), device="cuda")
            ft = torch.as_tensor(f[None], device="cuda").contiguous()
            ws.predict(ft)  # first call warms the kernels
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            xw = ws.predict(ft)[0]
            e1.record()
            torch.cuda.synchronize()
            fwd_ms.append(e0.elapsed_time(e1))
            cold = plan.run(xr, xr, **opts)
            warm = ws.run(plan, ft, xr, warm_alpha=args.warm_alpha, **opts)
            # reference: both starts run long at the floor step without the stop
            # rule; their traces give the updates each needs to come within 1e-3
            # of the best value
            ref_a = args.alpha_min if args.alpha_min > 0 else args.alpha
            ref_c = plan.run(None, xr, trace=True, x_best=True, max_iter=args.ref_iters,
                             alpha=ref_a)
            ref_w = plan.run(None, xw, trace=True, max_iter=args.ref_iters, alpha=ref_a)
            best = max(ref_c["trace_min"][-1], ref_w["trace_min"][-1],
                       1.0 / cold["sigma_min"], 1.0 / warm["sigma_min"])
            ub = ref_c["x_best_min"]
            overlap = float(abs(torch.dot(xw, ub)) / (xw.norm() * ub.norm()))

            def upd(tr):
                hit = np.nonzero(tr >= (1 - 1e-3) * best)[0]
                return int(hit[0]) + 1 if hit.size else None

            k_ref = cold["sigma_max"] * best
            k_cold = cold["kappa"]
            k_warm = cold["sigma_max"] / warm["sigma_min"]
            rows.append(dict(seed=seed, cold_iters=cold["iters_min"], cold_ms=cold["ms_min"],
                             warm_iters=warm["iters_warm"], warm_total_iters=warm["iters_total"],
                             warm_ms=warm["ms_min"], fallback=warm["fallback"],
                             kappa_ref=k_ref, kappa_plain=k_cold, kappa_warm=k_warm,
                             err_plain=(k_ref - k_cold) / k_ref, err_warm=(k_ref - k_warm) / k_ref,
                             kappa_rel_diff=abs(k_warm - k_cold) / k_cold, overlap=overlap,
                             updates_to_1e3_plain=upd(ref_c["trace_min"]),
                             updates_to_1e3_warm=upd(ref_w["trace_min"]),
                             sigma_max_ms=cold["ms_max"]))
            plan.close()
            r_ = rows[-1]
            print(f"[bench] test {i + 1}/{args.test_count}: stop rule: plain {cold['iters_min']} "
                  f"updates {cold['ms_min']:.0f} ms err {r_['err_plain']:.1e}; warm "
                  f"{warm['iters_warm']}+check {warm['ms_min']:.0f} ms err {r_['err_warm']:.1e} "
                  f"fallback {warm['fallback']}; to 1e-3 of the best: plain "
                  f"{r_['updates_to_1e3_plain']} warm {r_['updates_to_1e3_warm']}; overlap "
                  f"{overlap:.3f}", file=sys.stderr, flush=True)
    ws.close()
    cold_ms = np.array([r["cold_ms"] for r in rows])
    warm_ms = np.array([r["warm_ms"] for r in rows])
    smax_ms = np.array([r["sigma_max_ms"] for r in rows])
    # forward pass: 2 * 9 * sum(cin * cout) FLOP per node with the true channel counts
    flops = 2 * 9 * (2 * 64 + 64 * 64 + 64 * 64 + 64 * 6) * side * side
    fwd = float(np.median(fwd_ms))
    train_desc = " + ".join(f"{max(16, int(round(c * args.train_scale)))} {s}x{s}"
                            for s, c in w["train"])
    out = {
        "metric": "time-to-kappa (1e-3 rel) per matrix, warm-started vs plain",
        "value": float(np.mean(smax_ms + warm_ms)) / 1e3 + fwd / 1e3, "unit": "s", "n_gpus": 1,
        "steps": len(rows), "warmup": 0,
        "ms_per_step": float(np.mean(smax_ms + warm_ms)) + fwd, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (network bf16/f32)",
        "data": "synthetic",
        "config": {"workload": f"c5warm: held-out {side}x{side} hydro-mechanical systems "
                               f"(seeds {first}-{first + args.test_count - 1}), network trained "
                               f"on {train_desc} systems",
                   "epochs": args.epochs, "stop_rtol": args.stop_rtol,
                   "stop_window": args.stop_window, "parallelism": "single GPU"},
        "plain_s": float(np.mean(smax_ms + cold_ms)) / 1e3,
        "speedup_sigma_min": float(np.sum(cold_ms) / np.sum(warm_ms)),
        "fallback_rate": float(np.mean([r["fallback"] for r in rows])),
        "kappa_rel_diff_max": float(max(r["kappa_rel_diff"] for r in rows)),
        "kappa_err_max": {"plain": float(max(r["err_plain"] for r in rows)),
                          "warm": float(max(r["err_warm"] for r in rows))},
        "updates_to_1e3_median": {
            k: float(np.median([r[f"updates_to_1e3_{k}"] if r[f"updates_to_1e3_{k}"] is not None
                                else args.ref_iters + 1 for r in rows])) for k in ("plain", "warm")},
        "warm_alpha": args.warm_alpha,
        "overlap_median": float(np.median([r["overlap"] for r in rows])),
        "updates_median": {"plain": float(np.median([r["cold_iters"] for r in rows])),
                           "warm": float(np.median([r["warm_iters"] for r in rows])),
                           "warm_with_check": float(np.median([r["warm_total_iters"]
                                                               for r in rows]))},
        "forward": {"ms": fwd, "gflop": flops / 1e9,
                    "tflops": flops / (fwd * 1e-3) / 1e12},
        "roofline": {"bound": "mfma", "achieved": flops / (fwd * 1e-3) / 1e12, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": flops / (fwd * 1e-3) / 1e12 / 2500.0,
                     "traffic": None, "kernel": "cnn forward (prep + 4 convs + output)"},
        "label_s": label_s, "train_s": train_s, "loss": [hist[0], hist[-1]],
        "criterion": warm_criterion(rows, args.ref_iters),
        "tests": rows,
    }
    print(json.dumps(out), flush=True)


def warm_criterion(rows, ref_iters):
    """The warm-start criterion fixed before the evaluation: (1) the median
    over systems of the ratio of updates to 1e-3 of the best value found
    (predicted start / random start) and the share of systems where the
    predicted start is ahead; (2) the mean sigma_min time of the whole
    warm-started estimate over the plain run's; it pays iff (2) <= 1 with
    both estimates within 1e-3 of the best value found."""
    def upd(r, k):
        v = r[f"updates_to_1e3_{k}"]
        return v if v is not None else ref_iters + 1

    ratios = np.array([upd(r, "warm") / upd(r, "plain") for r in rows])
    t_ratio = float(np.mean([r["warm_ms"] for r in rows]) / np.mean([r["cold_ms"] for r in rows]))
    accurate = all(r["err_plain"] <= 1e-3 and r["err_warm"] <= 1e-3 for r in rows)
    return {"systems": len(rows), "median_update_ratio": float(np.median(ratios)),
            "share_ahead": float(np.mean(ratios < 1.0)), "time_ratio_warm_over_plain": t_ratio,
            "both_within_1e-3": accurate, "pays": bool(t_ratio <= 1.0 and accurate)}


def bench_batch(w, args):
    """Batched multi-start sigma_max run vs a loop of plain runs, same starts and options."""
    import torch

    import paper_2409_11515_amd as pa
    from synth import hm_batch_specs, hydromech2d, start_block

    t0 = time.perf_counter()
    specs = hm_batch_specs(count=w["count"], side_range=w["side_range"])
    mats = [hydromech2d(s, log_eta=le, log_k=lk) for s, le, lk in specs]
    starts = [start_block(m.n, 8, 7000 + i) for i, m in enumerate(mats)]
    gen_s = time.perf_counter() - t0
    nrows = sum(m.n for m in mats)
    nnz = sum(m.nnz for m in mats)
    print(f"[bench] batch: {len(mats)} matrices, rows {nrows}, nnz {nnz} ({gen_s:.0f}s)",
          file=sys.stderr, flush=True)
    opts = dict(max_iter=args.max_iter, stop_rtol=args.stop_rtol, stop_window=args.stop_window,
                alpha=args.alpha, alpha_min=args.alpha_min, alpha_decay=0.5)
    t0 = time.perf_counter()
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in mats], **opts).bind()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    x0 = torch.as_tensor(pa.interleave_starts(starts), device="cuda")
    for _ in range(args.warmup):
        b.run(x0)
    times = []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rb = b.run(x0)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"[bench] batched step {k}: {times[-1]*1e3:.1f} ms", file=sys.stderr, flush=True)
    batched_s = float(np.mean(times))
    # plain path: one plan per matrix, one run per start
    t_plain = 0.0
    max_rel = 0.0
    plain_iters = 0
    for i, m in enumerate(mats):
        p = pa.Plan(m.n, m.rowptr, m.col, m.val, sigma_min_method=pa.COND_MIN_NONE, **opts).bind()
        xs = [torch.as_tensor(starts[i][k], device="cuda") for k in range(8)]
        p.run(xs[0])  # warm the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best = [p.run(xs[k]) for k in range(8)]
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        plain_iters += sum(r["iters_max"] for r in best)
        smax = max(r["sigma_max"] for r in best)
        max_rel = max(max_rel, abs(smax - rb["sigma_max"][i]) / smax)
        p.close()
        if i % 16 == 15:
            print(f"[bench] plain loop: {i+1} matrices", file=sys.stderr, flush=True)
    b_iters = int(rb["pair_iters"].sum())
    b.close()
    kap = bench_batch_kappa(mats, starts, rb["sigma_max"], opts, args) if args.kappa_systems else None
    full = kap is not None and kap["systems"] == len(mats)
    value = (batched_s + kap["sigma_min_run_s"]) / len(mats) if full else batched_s / len(mats)
    out = {
        "metric": "time-to-kappa (1e-3 rel) per matrix + SpMV HBM GB/s",
        "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": batched_s * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c4batch: 64 hydro-mechanical matrices, sides U{51..401}, "
                               "8 starts each", "rows": nrows, "nnz": nnz,
                   "tile_rows": b.tile_rows, "grid": b.grid, "parallelism": "single GPU"},
        "value_is": ("batched sigma_max and sigma_min runs of every matrix (kappa), per matrix"
                     if full else "batched sigma_max run per matrix"),
        "batched_s": batched_s, "plain_loop_s": t_plain, "speedup": t_plain / batched_s,
        "pair_updates": {"batched": b_iters, "plain": plain_iters},
        "sigma_max_rel_diff_max": max_rel, "setup_s": setup_s,
        "kappa": kap,
    }
    print(json.dumps(out), flush=True)


def bench_batch_kappa(mats, starts_max, sigma_max, opts, args):
    """Batched sigma_min over the first `kappa_systems` matrices (every
    matrix's LU on the host in parallel threads, the solves of all of them
    and their 8 starts in one launch each), kappa per matrix, and the plain
    loop (one plan and LU per matrix, one sigma_min run per start) on a
    sample of them against a batch of the same sample."""
    import torch

    import paper_2409_11515_amd as pa
    from synth import start_block

    count = min(args.kappa_systems, len(mats))
    sub = mats[:count]
    starts = [start_block(m.n, 8, 9000 + i) for i, m in enumerate(sub)]
    t0 = time.perf_counter()
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in sub], sigma_min=True, **opts)
    create_s = time.perf_counter() - t0
    fill = b.fill()
    t0 = time.perf_counter()
    b.bind()
    torch.cuda.synchronize()
    bind_s = time.perf_counter() - t0
    print(f"[bench] batched sigma_min: {count} matrices, LU + schedules {create_s:.0f}s "
          f"(LU threads {fill['lu_s']:.0f}s), bind {bind_s:.0f}s, fill {fill['nnz_l'] + fill['nnz_u']:.3g}",
          file=sys.stderr, flush=True)
    x0 = torch.as_tensor(pa.interleave_starts(starts), device="cuda")
    b.run_min(x0, max_iter=30)  # capture the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rm = b.run_min(x0)
    torch.cuda.synchronize()
    min_s = time.perf_counter() - t0
    b.close()
    kappa = np.asarray(sigma_max[:count]) / rm["sigma_min"]
    print(f"[bench] batched sigma_min run {min_s:.1f}s, kappa {kappa.min():.3g}..{kappa.max():.3g}",
          file=sys.stderr, flush=True)
    # plain loop and a batch on a sample spread over the sizes
    order = np.argsort([m.n for m in sub])
    sample = sorted(int(order[k]) for k in np.linspace(0, count - 1, min(args.kappa_sample, count)).astype(int))
    smats = [sub[i] for i in sample]
    sb = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in smats], sigma_min=True, **opts).bind()
    sx0 = torch.as_tensor(pa.interleave_starts([starts[i] for i in sample]), device="cuda")
    sb.run_min(sx0, max_iter=30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = sb.run_min(sx0)
    torch.cuda.synchronize()
    sample_batched_s = time.perf_counter() - t0
    sb.close()
    t_plain = 0.0
    max_rel = 0.0
    plain_updates = 0
    for j, i in enumerate(sample):
        m = sub[i]
        p = pa.Plan(m.n, m.rowptr, m.col, m.val, **opts).bind()
        xs = [torch.as_tensor(starts[i][k], device="cuda") for k in range(8)]
        p.run(None, xs[0], max_iter=30)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [p.run(None, xs[k]) for k in range(8)]
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        plain_updates += sum(r["iters_min"] for r in res)
        smin = min(r["sigma_min"] for r in res)
        max_rel = max(max_rel, abs(smin - rs["sigma_min"][j]) / smin,
                      abs(smin - rm["sigma_min"][i]) / smin)
        p.close()
    print(f"[bench] sample of {len(sample)}: plain loop {t_plain:.1f}s, batched {sample_batched_s:.1f}s",
          file=sys.stderr, flush=True)
    return {"systems": count, "rows": int(sum(m.n for m in sub)),
            "fill": fill["nnz_l"] + fill["nnz_u"], "lu_threads_s": fill["lu_s"],
            "create_s": create_s, "bind_s": bind_s, "sigma_min_run_s": min_s,
            "pair_updates": int(rm["pair_iters"].sum()),
            "kappa_min": float(kappa.min()), "kappa_max": float(kappa.max()),
            "kappa_per_matrix_s": min_s / count,
            "sample": {"systems": sample, "sides": [int(round((m.n / 6) ** 0.5)) for m in smats],
                       "plain_loop_s": t_plain, "batched_s": sample_batched_s,
                       "speedup": t_plain / sample_batched_s, "plain_updates": plain_updates,
                       "batched_updates": int(rs["pair_iters"].sum()),
                       "sigma_min_rel_diff_max": max_rel}}


def make_matrix(w):
    from synth import hydromech2d, stokes2d

    if w["kind"] == "hm":
        return hydromech2d(w["side"], seed=w["seed"])
    return stokes2d(w["side"], w["side"], seed=w["seed"])


def _source_hash(kind):
    """SHA-256 of the code a kernel family's counters in profiles/pmc_traffic.json
    were taken on: for "trsv" the single-side triangular-solve section of
    kernels.hip and the single-matrix panel schedule in panels.cpp (the
    joining of several matrices' schedules, which only the batch uses, left
    out), for "spmv" the streaming SpMV section of kernels.hip and the row
    tiles in plan.hip."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2409_11515_amd", "csrc")
    with open(os.path.join(csrc, "kernels.hip")) as f:
        src = f.read()
    with open(os.path.join(csrc, "plan.hip")) as f:
        plan = f.read()
    if kind == "trsv":
        with open(os.path.join(csrc, "panels.cpp")) as f:
            panels = f.read()
        parts = [src[src.index("// ----------------------------------------------------------------- trsv"):
                     src.index("// ------------------------------------------------- trsv, several sides")],
                 panels[panels.index("constexpr int64_t kSliceEntries"):panels.index("PanelCsr merge_panels(")],
                 panels[panels.index("// The inverse of every panel's triangle"):panels.index("// Row i -> n-1-i")]]
    else:
        parts = [src[src.index("// ---------------------------------------------------------- spmv (stream)"):
                     src.index("// ---------------------------------------------------------------- sumsq")],
                 plan[plan.index("// Row tiles for the streaming SpMV"):plan.index("}  // namespace\n\nstruct cond_plan")]]
    return hashlib.sha256("".join(parts).encode()).hexdigest()


def pmc_traffic(workload, kernel, key):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (profiles/pmc_traffic.json), or None when they were taken on another
    version of the kernel's source, on other data (key: the fill of L and U
    for the solves, n and nnz for the SpMV) or not for this workload."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    wl = rec.get("workloads", {}).get(workload, {})
    if kernel not in wl:
        return None
    kind = "trsv" if kernel.startswith("trsv") else "spmv"
    if wl.get("source_sha256") != _source_hash(kind) or list(wl.get("key", [])) != list(key):
        return None
    return wl[kernel]["traffic_bytes"]


def golden(w):
    """(kappa the oracle reaches with the bench's options, a more accurate
    reference kappa) from tests/golden/, either None when not stored."""
    if not w["golden"]:
        return None, None
    path = os.path.join(ROOT, "tests", "golden", w["golden"])
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        g = json.load(f)
    if "kappa_svd" in g:  # exact (extended-precision SVD)
        return None, g["kappa_svd"]
    return g.get("kappa"), g.get("reference", {}).get("kappa")


def host_cpu():
    """CPU model and logical CPU count of this host (for the baseline's record)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(a, iters_max, iters_min, budget_s=25.0, min_route=True):
    """Oracle per-update times on a bounded sample, scaled to the GPU's update counts."""
    from oracle import PAOptions
    from oracle.estimate import forward_apply
    from oracle.inverse import LUInverse
    from oracle.padam import projected_adam
    from synth import start_vector

    x0 = start_vector(a.n, 11)
    apply_f, eval_f = forward_apply(a.n, a.rowptr, a.col, a.val)
    t0 = time.perf_counter()
    projected_adam(apply_f, eval_f, x0, PAOptions(max_iter=3))
    per_max = (time.perf_counter() - t0) / 4
    k_max = int(max(3, min(iters_max, 0.2 * budget_s / max(per_max, 1e-9))))
    t0 = time.perf_counter()
    projected_adam(apply_f, eval_f, x0, PAOptions(max_iter=k_max))
    per_max = (time.perf_counter() - t0) / (k_max + 1)
    host = host_cpu()
    where = f"1 of {host['logical_cpus']} cores ({host['model']}), one thread"
    if not min_route:
        return {
            "value": iters_max * per_max, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"{k_max} sigma_max updates of the oracle on the same matrix, scaled to "
                       f"the GPU's {iters_max} updates (sigma_max run only); {where}"),
            "per_update_ms": {"sigma_max": per_max * 1e3}, "host": host,
        }
    t0 = time.perf_counter()
    inv = LUInverse(a.n, a.rowptr, a.col, a.val)
    lu_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    projected_adam(inv.apply, inv.evaluate, start_vector(a.n, 12), PAOptions(max_iter=2))
    per_min = (time.perf_counter() - t0) / 3
    left = budget_s - lu_s - k_max * per_max
    k_min = int(max(2, min(iters_min, 0.8 * left / max(per_min, 1e-9))))
    t0 = time.perf_counter()
    projected_adam(inv.apply, inv.evaluate, start_vector(a.n, 12), PAOptions(max_iter=k_min))
    per_min = (time.perf_counter() - t0) / (k_min + 1)
    value = iters_max * per_max + iters_min * per_min
    return {
        "value": value, "unit": "s", "cores": 1, "kind": "oracle",
        "sample": (f"{k_max} sigma_max updates and {k_min} sigma_min updates of the oracle on "
                   f"the same matrix, scaled to the GPU's {iters_max} + {iters_min} updates; "
                   f"SuperLU factorisation ({lu_s:.1f} s) excluded like the GPU's host LU; "
                   f"{where}"),
        "per_update_ms": {"sigma_max": per_max * 1e3, "sigma_min": per_min * 1e3},
        "lu_s": lu_s, "host": host,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="hm201", choices=sorted(WORKLOADS))
    ap.add_argument("--max-iter", type=int, default=6000)
    ap.add_argument("--stop-rtol", type=float, default=1e-6)
    ap.add_argument("--stop-window", type=int, default=25)
    ap.add_argument("--alpha", type=float, default=None,
                    help="initial Adam step size (default: the workload's)")
    ap.add_argument("--alpha-min", type=float, default=2.5e-3,
                    help="step-size floor: on a plateau alpha halves down to this (0: constant alpha)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kappa-systems", type=int, default=64,
                    help="c4batch: matrices of the batched sigma_min run (0: sigma_max only)")
    ap.add_argument("--kappa-sample", type=int, default=6,
                    help="c4batch: matrices of the plain-loop comparison of the sigma_min run")
    ap.add_argument("--no-hbm-section", dest="hbm_section", action="store_false",
                    help="skip the streaming ceiling and the 1001x1001 SpMV roofline section")
    ap.add_argument("--train-scale", type=float, default=1.0,
                    help="c5warm: multiplies the training-set sizes")
    ap.add_argument("--test-count", type=int, default=8, help="c5warm: held-out matrices")
    ap.add_argument("--test-first", type=int, default=0,
                    help="c5warm: index of the first held-out matrix (seed 20000 + index)")
    ap.add_argument("--epochs", type=int, default=60, help="c5warm: training epochs")
    ap.add_argument("--params-in", default=None, help="c5warm: trained parameters (.npy), no training")
    ap.add_argument("--params-out", default=None, help="c5warm: save the trained parameters (.npy)")
    ap.add_argument("--warm-alpha", type=float, default=1e-2, help="c5warm: alpha of the warm run")
    ap.add_argument("--ref-iters", type=int, default=2500,
                    help="c5warm: updates of the long reference runs without the stop rule")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2409_11515_amd as pa
    from synth import start_vector

    w = WORKLOADS[args.workload]
    if args.alpha is None:
        args.alpha = w["alpha"]
    if w["kind"] == "batch":
        bench_batch(w, args)
        return
    if w["kind"] == "warm":
        bench_warm(w, args)
        return
    t0 = time.perf_counter()
    a = make_matrix(w)
    gen_s = time.perf_counter() - t0
    print(f"[bench] workload {args.workload}: n={a.n} nnz={a.nnz} (generated in {gen_s:.1f}s)",
          file=sys.stderr, flush=True)
    opts = dict(max_iter=args.max_iter, stop_rtol=args.stop_rtol, stop_window=args.stop_window,
                alpha=args.alpha, alpha_min=args.alpha_min, alpha_decay=0.5,
                sigma_min_method=pa.COND_MIN_LU if w["min_route"] else pa.COND_MIN_NONE)
    t0 = time.perf_counter()
    plan = pa.Plan(a.n, a.rowptr, a.col, a.val, **opts)
    plan.bind()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"[bench] plan ready in {setup_s:.1f}s (workspace {plan.workspace_bytes/2**20:.0f} MiB)",
          file=sys.stderr, flush=True)
    x0a = torch.as_tensor(start_vector(a.n, 11), device="cuda")
    x0b = torch.as_tensor(start_vector(a.n, 12), device="cuda")
    for _ in range(args.warmup):
        plan.run(x0a, x0b)
    torch.cuda.synchronize()
    times = []
    res = None
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.run(x0a, x0b)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"[bench] step {k}: {times[-1]*1e3:.1f} ms kappa={res['kappa']:.6e} "
              f"sigma_max={res['sigma_max']:.6e} "
              f"iters={res['iters_max']}/{res['iters_min']}", file=sys.stderr, flush=True)
    step_s = float(np.mean(times))

    # time to the first 1e-3 crossing of the running kappa: the runs are
    # deterministic, so a traced repeat of the timed run gives the update at
    # which sigma_max (final: its run ends first) times the running best
    # ||A^-1 x|| first comes within 1e-3 of the reference kappa; the time is
    # the timed sigma_max run plus that share of the timed sigma_min run
    gk, gref = golden(w)
    kref = gk if gk else gref
    crossing = None
    if w["min_route"]:
        tr = plan.run(x0a, x0b, trace=True)
        assert tr["kappa"] == res["kappa"], "traced repeat differs from the timed run"
        ref = kref if kref else res["kappa"]
        kap = tr["sigma_max"] * np.asarray(tr["trace_min"])
        hit = np.nonzero(np.abs(kap / ref - 1.0) <= 1e-3)[0]
        if hit.size:
            t_hit = int(hit[0]) + 1
            frac = t_hit / (res["iters_min"] + 1)
            crossing = {"update": t_hit, "of": res["iters_min"],
                        # the timed step apportioned by the two runs' device times
                        "s": step_s * (res["ms_max"] + frac * res["ms_min"])
                        / (res["ms_max"] + res["ms_min"]),
                        "reference": "oracle, same starts and options" if kref == gk and gk
                        else ("extended-precision SVD" if kref else "the run's own final kappa")}

    # Algorithm 1 as the paper writes it (constant step, no floor) at a step
    # small enough to reach 1e-3: the plain baseline beside the schedule
    const = None
    if w["min_route"] and args.alpha_min > 0:
        a_c = args.alpha_min
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = plan.run(x0a, x0b, alpha=a_c, alpha_min=0.0)
        torch.cuda.synchronize()
        const = {"alpha": a_c, "s": time.perf_counter() - t0, "kappa": rc["kappa"],
                 "iters": {"sigma_max": rc["iters_max"], "sigma_min": rc["iters_min"]},
                 "kappa_rel_err": (abs(rc["kappa"] - kref) / kref) if kref else None}

    # profiled run: per-kernel average durations from HIP events
    prof = plan.run(x0a, x0b, profile=1)
    stats = plan.kernel_stats()
    dom = max(stats, key=lambda k: stats[k][0])
    ms_tot, cnt, byts = stats[dom]
    avg_ms = ms_tot / max(cnt, 1)
    achieved = byts / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    kernels = {k: {"avg_us": (v[0] / v[1] * 1e3) if v[1] else None, "launches": v[1],
                   "alg_bytes": v[2],
                   "gbs": (v[2] / (v[0] / v[1] * 1e-3) / 1e9) if v[1] and v[0] > 0 else None}
               for k, v in stats.items() if v[1]}
    spmv = kernels.get("spmv_A")

    traffic_key = [res["nnz_l"], res["nnz_u"]] if dom.startswith("trsv") else [a.n, a.nnz]
    out = {
        "metric": "time-to-kappa (1e-3 rel) per matrix + SpMV HBM GB/s",
        "value": crossing["s"] if crossing else step_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: six-field staggered-grid hydro-mechanical matrix"
                               if w["kind"] == "hm" else "tiny Stokes",
                   "n": a.n, "nnz": a.nnz, "nnz_l": res["nnz_l"], "nnz_u": res["nnz_u"],
                   "alpha": args.alpha, "alpha_min": args.alpha_min, "max_iter": args.max_iter,
                   "stop_rtol": args.stop_rtol, "stop_window": args.stop_window,
                   "parallelism": "single GPU"},
        "kappa": res["kappa"] if w["min_route"] else None,
        "sigma_max": res["sigma_max"],
        "runs": "sigma_max and sigma_min" if w["min_route"] else "sigma_max only",
        "kappa_golden": gk,
        "kappa_rel_err": (abs(res["kappa"] - gk) / gk) if gk else None,
        "kappa_reference": gref,
        "kappa_reference_err": (abs(res["kappa"] - gref) / gref) if gref else None,
        "iters": {"sigma_max": res["iters_max"], "sigma_min": res["iters_min"]},
        "run_ms": {"sigma_max": res["ms_max"], "sigma_min": res["ms_min"]},
        "value_is": ("time to the first 1e-3 crossing of the running kappa" if crossing
                     else "time of the whole estimate (both runs to the stop rule)"),
        "time_to_stop_rule_s": step_s,
        "first_crossing": crossing,
        "setup_s": setup_s,
        "end_to_end_s": setup_s + step_s,
        "constant_alpha": const,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": pmc_traffic(args.workload, dom, traffic_key),
                     "kernel": dom, "avg_us": avg_ms * 1e3, "alg_bytes_per_launch": byts},
        "spmv": spmv,
        "kernels": kernels,
    }
    if w["min_route"]:
        # panel schedule of each triangular solve: (dependency levels, tasks, panels)
        out["trsv_schedule"] = {k: dict(zip(("levels", "tasks", "panels"), v))
                                for k, v in plan.solve_info().items()}
    plan.close()
    if args.hbm_section:
        out["stream_triad"] = stream_ceiling()
        out["hm1001_sigma_max"] = hm1001_section(out["stream_triad"]["gbs"])
        tri = out["stream_triad"]["gbs"]
        out["roofline"]["frac_of_triad"] = achieved / tri
        for k in out["kernels"].values():
            if k.get("gbs"):
                k["frac_of_triad"] = k["gbs"] / tri
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a, res["iters_max"], res["iters_min"],
                                           min_route=w["min_route"])
    print(json.dumps(out), flush=True)


def stream_ceiling():
    """The library's streaming triad over 3 x 2 GiB (24 B per element)."""
    import paper_2409_11515_amd as pa

    best = None
    for grid in (8192, 32768, 65536):
        r = pa.stream_triad(1 << 28, grid=grid, reps=20)
        if best is None or r["gbs"] > best[0]["gbs"]:
            best = (r, grid)
    r, grid = best
    print(f"[bench] stream triad: {r['gbs']:.0f} GB/s ({grid} blocks)", file=sys.stderr, flush=True)
    return {"gbs": r["gbs"], "ms": r["ms"], "bytes": r["bytes"], "peak_frac": r["gbs"] / HBM_PEAK_GBS,
            "kernel": f"a = b + s c over 3 x 2 GiB, 16-byte accesses, 4 in flight per thread, "
                      f"best of 8192 / 32768 / 65536 blocks of 256 threads: {grid}"}


def hm1001_section(triad_gbs):
    """The HBM roofline measurement of the 6M-row system: a profiled stretch of
    its sigma_max run (its sigma_min run needs a host LU of about 1.2e9
    entries, beyond this benchmark's time)."""
    import torch

    import paper_2409_11515_amd as pa
    from synth import hydromech2d, start_vector

    t0 = time.perf_counter()
    a = hydromech2d(1001, seed=2)
    p = pa.Plan(a.n, a.rowptr, a.col, a.val, sigma_min_method=pa.COND_MIN_NONE).bind()
    gen = time.perf_counter() - t0
    x0 = torch.as_tensor(start_vector(a.n, 11), device="cuda")
    p.run(x0, max_iter=40, alpha=4e-2)
    p.run(x0, max_iter=60, alpha=4e-2, profile=1)
    stats = p.kernel_stats()
    p.close()
    ks = {}
    for k, (ms, cnt, byts) in stats.items():
        if cnt:
            gbs = byts / (ms / cnt * 1e-3) / 1e9
            ks[k] = {"avg_us": ms / cnt * 1e3, "launches": cnt, "alg_bytes": byts, "gbs": gbs,
                     "frac": gbs / HBM_PEAK_GBS, "frac_of_triad": gbs / triad_gbs}
    print(f"[bench] hm1001 sigma_max section ({gen:.0f}s set-up): "
          + ", ".join(f"{k} {v['gbs']:.0f} GB/s" for k, v in ks.items()), file=sys.stderr, flush=True)
    return {"n": a.n, "nnz": a.nnz, "updates_profiled": 60, "kernels": ks,
            "traffic_spmv_A": pmc_traffic("hm1001", "spmv_A", [a.n, a.nnz])}


if __name__ == "__main__":
    main()
