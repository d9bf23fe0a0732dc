"""Learned warm start for the sigma_min run (Algorithm 2), on the device.

The sigma_min run maximises ||A^-1 x|| / ||x||; any start converges to the
same maximiser, so a start that already points near it saves updates and
changes nothing else. ``WarmStart`` wraps the ``cond_cnn_*`` network:

* ``label``: plain sigma_min runs (random starts) on training matrices give
  the maximisers u, the network's targets;
* ``fit``: Adam on the sign- and scale-invariant loss 1 - (p.u)^2/(|p|^2|u|^2);
* ``run``: predicts x0 from the coefficient fields, runs the sigma_min
  iteration from it and, as the fallback, from a random start too, and keeps
  the larger ||A^-1 x|| / ||x|| (both are lower bounds of ||A^-1||, so the
  larger is never worse).

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

    def predict(self, fields):
        return self.net.predict(fields)

    def run(self, plan: Plan, fields, x0_random, x0_max=None, **opts) -> dict:
        """sigma_min from the predicted start and from x0_random; the result
        with the larger best (smaller sigma_min) wins. fields: [1, 2, s-1, s-1]."""
        x_warm = self.predict(fields)[0]
        x_max = x0_random if x0_max is None else x0_max
        warm = plan.run(x_max, x_warm, **opts)
        cold = plan.run(x_max, x0_random, **opts)
        out = dict(warm)
        out["fallback"] = cold["sigma_min"] < warm["sigma_min"]
        if out["fallback"]:
            out.update({k: cold[k] for k in ("sigma_min", "iters_min", "status_min")})
        out["kappa"] = out["sigma_max"] / out["sigma_min"]
        out["iters_min_warm"] = warm["iters_min"]
        out["iters_min_cold"] = cold["iters_min"]
        out["ms_min_warm"] = warm["ms_min"]
        out["ms_min_cold"] = cold["ms_min"]
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
