"""Oracle for the learned warm start: a small CNN, plain float64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network maps the two coefficient fields of a hydro-mechanical grid to a
start vector for the sigma_min run: four 3x3 "same" convolutions,
2 -> 64 -> 64 -> 64 -> 6 channels, ReLU after the first three, no activation
after the last. The six output channels of node (i, j) are the six unknowns
of that node, in the matrix's node-major order. The paper has no such
network; it is this project's warm start and changes nothing in the
estimator's arithmetic.

Precision model of the GPU kernels, mirrored here so that the oracle sees the
same rounded operands: weights and activations are bfloat16 (round to
nearest even), products are summed exactly here (float64) and in float32 on
the device, biases and the last layer's output are float32/float64.

Training loss per sample (sign-invariant, scale-invariant):
    l(p, u) = 1 - (p.u)^2 / ((p.p)(u.u))
with p the network output and u the minimiser found by the plain method.
"""

from __future__ import annotations

import numpy as np

CHANNELS = (2, 64, 64, 64, 6)
INPUT_SCALE = ((21.0, 3.0), (-16.0, 4.0))  # (centre, half-width) of log10 eta, log10 k


def bf16(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = rounded.astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, f, out)
    return out.astype(np.float64)


def node_fields(log_eta, log_k):
    """Cell fields (s-1, s-1) -> normalised node fields (2, s, s).

    A node takes the mean of its adjacent cells (edge cells replicated), then
    each field is centred and scaled to about [-1, 1].
    """
    out = []
    for f, (c, h) in zip((log_eta, log_k), INPUT_SCALE):
        p = np.pad(np.asarray(f, np.float64), 1, mode="edge")
        node = 0.25 * (p[:-1, :-1] + p[1:, :-1] + p[:-1, 1:] + p[1:, 1:])
        out.append((node - c) / h)
    return np.stack(out)


def init_params(seed: int = 0):
    """He-normal weights (3, 3, cin, cout) and zero biases, float64."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        w = rng.standard_normal((3, 3, cin, cout)) * np.sqrt(2.0 / (9 * cin))
        params.append((w, np.zeros(cout)))
    return params


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten(vec):
    params, off = [], 0
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        nw = 9 * cin * cout
        w = np.asarray(vec[off:off + nw], np.float64).reshape(3, 3, cin, cout)
        off += nw
        b = np.asarray(vec[off:off + cout], np.float64)
        off += cout
        params.append((w, b))
    return params


def conv3x3(x, w, b=None):
    """y[co, i, j] = b[co] + sum_{ky,kx,ci} x[ci, i+ky-1, j+kx-1] w[ky, kx, ci, co] (zero pad)."""
    c, h, wd = x.shape
    xp = np.zeros((c, h + 2, wd + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[3], h, wd))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + h, kx:kx + wd]  # (ci, h, w)
            y += np.tensordot(w[ky, kx], patch, axes=([0], [0]))  # (co, h, w)
    if b is not None:
        y += b[:, None, None]
    return y


def conv3x3_loops(x, w, b=None):
    """The same convolution written as its definition, for tiny inputs."""
    c, h, wd = x.shape
    co = w.shape[3]
    y = np.zeros((co, h, wd))
    for o in range(co):
        for i in range(h):
            for j in range(wd):
                s = 0.0 if b is None else b[o]
                for ky in range(3):
                    for kx in range(3):
                        ii, jj = i + ky - 1, j + kx - 1
                        if 0 <= ii < h and 0 <= jj < wd:
                            for ci in range(c):
                                s += x[ci, ii, jj] * w[ky, kx, ci, o]
                y[o, i, j] = s
    return y


def forward(params, x, rounded=True):
    """Activations of every layer; ``rounded`` applies the bfloat16 points."""
    r = bf16 if rounded else (lambda t: t)
    acts = [r(x)]
    for li, (w, b) in enumerate(params):
        z = conv3x3(acts[-1], r(w), b)
        if li < len(params) - 1:
            acts.append(r(np.maximum(z, 0.0)))
        else:
            acts.append(z)  # last layer stays in high precision
    return acts


def output_vector(out):
    """(6, s, s) network output -> start vector in node-major order 6*(i*s + j) + f."""
    return np.ascontiguousarray(np.transpose(out, (1, 2, 0)).reshape(-1))


def loss_and_grad(p, u):
    """l = 1 - (p.u)^2/((p.p)(u.u)) and dl/dp."""
    pu = p @ u
    pp = p @ p
    uu = u @ u
    loss = 1.0 - pu * pu / (pp * uu)
    grad = -2.0 * pu / (pp * uu) * u + 2.0 * pu * pu / (pp * pp * uu) * p
    return loss, grad


def backward(params, acts, dout, rounded=True):
    """Gradients (dW, db) of every layer given dl/d(output) of shape (6, s, s).

    The gradient flowing into each layer's output is rounded to bfloat16 as
    on the device (the last layer's incoming gradient included).
    """
    r = bf16 if rounded else (lambda t: t)
    grads = [None] * len(params)
    g = r(dout)
    for li in range(len(params) - 1, -1, -1):
        w, _ = params[li]
        wr = r(w)
        xin = acts[li]
        c, h, wd = xin.shape
        xp = np.zeros((c, h + 2, wd + 2))
        xp[:, 1:-1, 1:-1] = xin
        dw = np.zeros_like(w)
        for ky in range(3):
            for kx in range(3):
                patch = xp[:, ky:ky + h, kx:kx + wd]  # (ci, h, w)
                dw[ky, kx] = np.tensordot(patch, g, axes=([1, 2], [1, 2]))  # (ci, co)
        db = g.sum(axis=(1, 2))
        grads[li] = (dw, db)
        if li > 0:
            # d input = full correlation with the flipped kernel, then the ReLU mask
            wf = wr[::-1, ::-1].transpose(0, 1, 3, 2)  # (ky, kx, co, ci)
            dx = conv3x3(g, wf)
            g = r(dx * (xin > 0))
    return grads


def adam_step(vec, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on flat float64 parameters (returns new vec, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return vec - lr * mh / (np.sqrt(vh) + eps), m, v
