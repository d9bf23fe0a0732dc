"""Learned warm start for the sigma_min run (Algorithm 2), on the device.

The sigma_min run maximises ||A^-1 x|| / ||x||; any start converges to the
same maximiser, so a start that already points near it saves updates and
changes nothing else. ``WarmStart`` wraps the ``cond_cnn_*`` network:

* ``label``: plain sigma_min runs (random starts) on training matrices give
  the maximisers u, the network's targets;
* ``fit``: Adam on the sign- and scale-invariant loss 1 - (p.u)^2/(|p|^2|u|^2);
* ``run``: predicts x0 from the coefficient fields, runs the sigma_min
  iteration from it, gives a random start as many updates, and falls back to
  the random start when that one reached the larger ||A^-1 x|| / ||x||
  (both are lower bounds of ||A^-1||, so the larger is never worse).

Every step runs in the library's kernels; this module only moves arguments.
"""

from __future__ import annotations

import numpy as np

from . import CNN, COND_MIN_LU, Plan


def label(plan: Plan, x0, **opts):
    """The best sigma_min iterate of a plain run from x0 (device float64),
    normalised, as float32 on the device; plus the run's result."""
    import torch

    r = plan.run(x0, x0, x_best=True, **opts)
    u = r["x_best_min"]
    return (u / u.norm()).to(torch.float32), r


class WarmStart:
    """The network plus its training loop and the warm-started run."""

    def __init__(self, max_batch: int, max_side: int, params=None, train=True, seed=0):
        self.net = CNN(max_batch, max_side, train=train)
        if params is None:
            params = init_params(seed)
        self.net.set_params(params)

    def params(self) -> np.ndarray:
        return self.net.get_params()

    def fit(self, fields, labels, epochs: int, batch: int, lr: float = 1e-3, seed: int = 0,
            lr_final: float | None = None, log=None) -> list:
        """Adam over shuffled mini-batches of one side. fields: CUDA float64
        [N, 2, s-1, s-1]; labels: CUDA float32 [N, 6 s^2]. Returns the mean
        loss of every epoch. With lr_final the rate decays geometrically."""
        import torch

        n = int(fields.shape[0])
        rng = np.random.default_rng(seed)
        steps = epochs * max(1, n // batch)
        decay = 1.0 if lr_final is None else (lr_final / lr) ** (1.0 / max(1, steps - 1))
        rate = lr
        history = []
        for ep in range(epochs):
            order = rng.permutation(n)
            tot, cnt = 0.0, 0
            for i in range(0, n - batch + 1, batch):
                idx = torch.as_tensor(order[i:i + batch], device=fields.device)
                tot += self.net.train_step(fields.index_select(0, idx).contiguous(),
                                           labels.index_select(0, idx).contiguous(), rate)
                cnt += 1
                rate *= decay
            history.append(tot / max(cnt, 1))
            if log:
                log(f"epoch {ep + 1}/{epochs} loss {history[-1]:.4f}")
        return history

    def fit_sets(self, sets, epochs: int, batch: int, lr: float = 1e-3, seed: int = 0,
                 lr_final: float | None = None, log=None) -> list:
        """Adam over training sets of different sides, [(fields, labels), ...]
        as in fit; every epoch visits the mini-batches of all sets in one
        shuffled order (each mini-batch holds one side)."""
        import torch

        rng = np.random.default_rng(seed)
        steps_per_epoch = sum(max(1, int(f.shape[0]) // batch) for f, _ in sets)
        steps = epochs * steps_per_epoch
        decay = 1.0 if lr_final is None else (lr_final / lr) ** (1.0 / max(1, steps - 1))
        rate = lr
        history = []
        for ep in range(epochs):
            work = []
            for k, (f, _) in enumerate(sets):
                order = rng.permutation(int(f.shape[0]))
                work += [(k, order[i:i + batch]) for i in range(0, len(order) - batch + 1, batch)]
            tot = 0.0
            for w in rng.permutation(len(work)):
                k, idx = work[w]
                f, lab = sets[k]
                ti = torch.as_tensor(idx, device=f.device)
                tot += self.net.train_step(f.index_select(0, ti).contiguous(),
                                           lab.index_select(0, ti).contiguous(), rate)
                rate *= decay
            history.append(tot / max(len(work), 1))
            if log:
                log(f"epoch {ep + 1}/{epochs} loss {history[-1]:.4f}")
        return history

    def predict(self, fields):
        return self.net.predict(fields)

    def run(self, plan: Plan, fields, x0_random, warm_alpha=None, **opts) -> dict:
        """The sigma_min run from the predicted start, with a random start as
        the fallback. fields: CUDA float64 [1, 2, s-1, s-1]. warm_alpha, if
        given, is the step size of the run from the predicted start (a start
        close to the maximiser survives only steps small against its entries);
        the random-start runs use the options as given.

        1. Run from the predicted start until the stop rule (or max_iter).
        2. Give the random start the same number of updates (the check).
        3. If the check reached a larger ||A^-1 x|| / ||x||, the prediction was
           worse than chance: run the random start to the stop rule and keep
           that result (the fallback).
        Returns sigma_min, the updates and device milliseconds spent in all
        runs together, and whether the fallback was taken."""
        x_warm = self.predict(fields)[0]
        warm = plan.run(None, x_warm, **({**opts, "alpha": warm_alpha} if warm_alpha else opts))
        t = max(1, int(warm["iters_min"]))
        check = plan.run(None, x0_random, **{**opts, "max_iter": t})
        out = dict(sigma_min=warm["sigma_min"], iters_warm=t, iters_total=t + check["iters_min"],
                   ms_min=warm["ms_min"] + check["ms_min"], fallback=False,
                   status_min=warm["status_min"])
        if check["sigma_min"] < warm["sigma_min"]:
            cold = plan.run(None, x0_random, **opts)
            out.update(sigma_min=cold["sigma_min"], fallback=True, status_min=cold["status_min"],
                       iters_total=out["iters_total"] + cold["iters_min"],
                       ms_min=out["ms_min"] + cold["ms_min"])
        return out

    def close(self):
        self.net.close()


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, float32, in the library's parameter order."""
    rng = np.random.default_rng(seed)
    chans = (2, 64, 64, 64, 6)
    parts = []
    for cin, cout in zip(chans[:-1], chans[1:]):
        parts.append(rng.standard_normal(9 * cin * cout) * np.sqrt(2.0 / (9 * cin)))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


__all__ = ["WarmStart", "label", "init_params", "COND_MIN_LU"]
