"""Warm-start CNN on the device against the CNN oracle (oracle/cnn.py).

Both sides round the same operands to bfloat16 (weights, activations, the
gradient entering each layer); the device sums products in float32 where the
oracle sums exactly. The input layer is therefore bit-exact. A float32 sum of
K <= 576 products differs from the exact one by at most about K 2^-24 of the
sum of magnitudes, so a stored activation differs by at most one bfloat16 ulp
(2^-7 of its value) wherever that bound stays below half an ulp, and such
flips are rare; after them the layers differ normwise by far less than the
bfloat16 rounding itself moves the result, which is what the tolerances
below check (each is stated beside its assertion).
"""

import numpy as np
import pytest

from oracle import cnn
from synth import hm_fields

pytestmark = pytest.mark.gpu

BF16_ULP = 2.0**-7  # largest relative spacing of bfloat16 numbers


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2409_11515_amd as pa

    pa._binding.lib()
    return torch


def _params(seed):
    rng = np.random.default_rng(seed)
    params = cnn.init_params(seed)
    # non-zero biases so that the bias paths are exercised; float32 masters
    params = [(w.astype(np.float32).astype(np.float64),
               (0.1 * rng.standard_normal(b.shape)).astype(np.float32).astype(np.float64))
              for w, b in params]
    return params


def _fields(side, seeds):
    cells = np.stack([np.stack(hm_fields(side, s)) for s in seeds])  # [B, 2, s-1, s-1]
    return np.ascontiguousarray(cells)


def _oracle_forward(params, cells, rounded=True):
    return [cnn.forward(params, cnn.node_fields(c[0], c[1]), rounded=rounded) for c in cells]


def _nhwc(a):  # (c, s, s) -> (s, s, c)
    return np.transpose(a, (1, 2, 0))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# 201: the full size of the warm-start workload (40401 pixels, a ragged last tile)
@pytest.mark.parametrize("side,seeds", [(13, (1, 2, 3)), (4, (7,)), (37, (5, 6)), (201, (9,))])
def test_forward_matches_oracle(torch_cuda, side, seeds):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    params = _params(11)
    cells = _fields(side, seeds)
    B = len(seeds)
    net = pa.CNN(max_batch=4, max_side=max(side, 40), train=False).set_params(cnn.flatten(params))
    x0 = net.predict(torch.as_tensor(cells, device="cuda")).cpu().numpy()
    ref = _oracle_forward(params, cells)
    unr = _oracle_forward(params, cells, rounded=False)
    for layer in range(5):
        got = net.activation(layer, B, side)
        want = np.stack([_nhwc(r[layer]) for r in ref])
        real = got[..., :want.shape[-1]]
        assert np.all(got[..., want.shape[-1]:] == 0.0)  # padded channels stay zero
        if layer == 0:
            np.testing.assert_array_equal(real, want)  # same rounding of the same value
        elif layer == 1:
            # one accumulation away from identical inputs: at most one ulp apart,
            # and almost all entries identical
            tol = BF16_ULP * np.abs(want) + 1e-6 * np.abs(want).max()
            assert np.all(np.abs(real - want) <= tol)
            assert np.mean(real != want) < 0.02
        else:
            gap = _rel(np.stack([_nhwc(u[layer]) for u in unr]), want)
            # differences from flipped roundings stay well below the rounding itself
            assert _rel(real, want) <= max(0.25 * gap, 1e-5), (layer, _rel(real, want), gap)
    want_x0 = np.stack([cnn.output_vector(r[-1]) for r in ref])
    assert _rel(x0, want_x0) <= 2e-3
    net.close()


def _oracle_gradients(params, cells, labels):
    B = len(cells)
    total = None
    losses = []
    for c, u in zip(cells, labels):
        acts = cnn.forward(params, cnn.node_fields(c[0], c[1]), rounded=True)
        l, gp = cnn.loss_and_grad(cnn.output_vector(acts[-1]), u.astype(np.float64))
        losses.append(l)
        s = acts[-1].shape[1]
        dout = np.transpose((gp / B).reshape(s, s, 6), (2, 0, 1))
        g = cnn.flatten(cnn.backward(params, acts, dout, rounded=True))
        total = g if total is None else total + g
    return total, np.array(losses)


def _layer_slices():
    out, off = [], 0
    for cin, cout in zip(cnn.CHANNELS[:-1], cnn.CHANNELS[1:]):
        out.append(slice(off, off + 9 * cin * cout))
        out.append(slice(off + 9 * cin * cout, off + 9 * cin * cout + cout))
        off += 9 * cin * cout + cout
    return out


def _labels(side, seeds, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((len(seeds), 6 * side * side)).astype(np.float32))


@pytest.mark.parametrize("side,seeds", [(13, (1, 2, 3)), (21, (4,)), (201, (9,))])
def test_gradients_match_oracle(torch_cuda, side, seeds):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    params = _params(12)
    cells = _fields(side, seeds)
    labels = _labels(side, seeds, 3)
    net = pa.CNN(max_batch=4, max_side=max(side, 32), train=True).set_params(cnn.flatten(params))
    g, losses = net.gradients(torch.as_tensor(cells, device="cuda"),
                              torch.as_tensor(labels, device="cuda"))
    g_ref, l_ref = _oracle_gradients(params, cells, labels)
    # the loss is a ratio of sums over the float32 output: relative 1e-5
    np.testing.assert_allclose(losses, l_ref, rtol=1e-5)
    # per layer (weights, then biases), normwise: the bfloat16 gradient chain
    # differs only by flipped roundings, a few parts in 1e3 at most
    for k, sl in enumerate(_layer_slices()):
        assert _rel(g[sl], g_ref[sl]) <= 1e-2, (k, _rel(g[sl], g_ref[sl]))
    net.close()


def test_gradients_are_deterministic(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    side, seeds = 19, (1, 2)
    cells = torch.as_tensor(_fields(side, seeds), device="cuda")
    labels = torch.as_tensor(_labels(side, seeds, 4), device="cuda")
    net = pa.CNN(max_batch=2, max_side=19).set_params(cnn.flatten(_params(3)))
    g1, l1 = net.gradients(cells, labels)
    g2, l2 = net.gradients(cells, labels)
    np.testing.assert_array_equal(g1, g2)
    np.testing.assert_array_equal(l1, l2)
    net.close()


def test_adam_step_matches_oracle(torch_cuda):
    """One Adam step on the device against the oracle's step from the oracle's
    gradient. On the first step the update is lr * g / (|g| + eps), which is
    lr times the sign of g wherever |g| >> eps: compare where the two
    gradients agree in sign with margin (all but a few tiny entries)."""
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    side, seeds = 15, (2, 3)
    params = _params(5)
    vec = cnn.flatten(params)
    cells = _fields(side, seeds)
    labels = _labels(side, seeds, 6)
    net = pa.CNN(max_batch=2, max_side=side).set_params(vec)
    lr = 1e-3
    ml = net.train_step(torch.as_tensor(cells, device="cuda"), torch.as_tensor(labels, device="cuda"),
                        lr)
    new = net.get_params().astype(np.float64)
    g_ref, l_ref = _oracle_gradients(params, cells, labels)
    assert ml == pytest.approx(l_ref.mean(), rel=1e-5)
    want, _, _ = cnn.adam_step(vec, g_ref, np.zeros_like(vec), np.zeros_like(vec), 1, lr=lr)
    sure = np.abs(g_ref) > 0.05 * np.abs(g_ref).max()
    assert sure.mean() > 0.05
    # float32 master weights: the step itself is exact to float32 rounding
    np.testing.assert_allclose(new[sure], want[sure], rtol=0, atol=4e-7 * np.abs(vec).max() + 1e-9)
    # every entry moved by at most lr (first Adam step) plus float32 rounding
    assert np.all(np.abs(new - vec.astype(np.float32)) <= lr * (1 + 1e-6) + 1e-6 * np.abs(vec))
    net.close()


def test_training_reduces_the_loss(torch_cuda):
    """Fit one fixed batch: the loss must fall well below its start."""
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    side, seeds = 17, (1, 2, 3, 4)
    cells = torch.as_tensor(_fields(side, seeds), device="cuda")
    # labels: a smooth function of the node fields, learnable by the network
    lab = []
    for s in seeds:
        le, lk = hm_fields(side, s)
        f = cnn.node_fields(le, lk)
        v = np.stack([f[0], f[1], f[0] * f[1], np.maximum(f[0], 0), f[1] ** 2, np.ones_like(f[0])])
        lab.append(cnn.output_vector(v))
    labels = torch.as_tensor(np.asarray(lab, np.float32), device="cuda")
    net = pa.CNN(max_batch=4, max_side=side).set_params(cnn.flatten(cnn.init_params(0)))
    first = net.train_step(cells, labels, 1e-3)
    for _ in range(150):
        last = net.train_step(cells, labels, 1e-3)
    assert last < 0.2 * first, (first, last)
    net.close()


def test_errors(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    net = pa.CNN(max_batch=2, max_side=9, train=False).set_params(cnn.flatten(_params(1)))
    cells = torch.as_tensor(_fields(9, (1, 2, 3)), device="cuda")
    with pytest.raises(pa.CondError):
        net.predict(cells)  # batch 3 > 2
    with pytest.raises(pa.CondError):
        net.gradients(cells[:2], torch.zeros(2, 6 * 81, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        net.set_params(np.zeros(10, np.float32))
    big = torch.as_tensor(_fields(11, (1,)), device="cuda")
    with pytest.raises(pa.CondError):
        net.predict(big)  # side 11 > 9
    net.close()
