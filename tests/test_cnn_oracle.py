"""Pins of the CNN oracle (oracle/cnn.py) on the CPU.

The convolution is checked against its definition written out as loops, the
backward pass against central finite differences, the loss against its
invariances, bfloat16 rounding against torch's conversion, and the first Adam
step against its closed form.
"""

import numpy as np
import pytest

from oracle import cnn


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 4))
    w = rng.standard_normal((3, 3, 3, 2))
    b = rng.standard_normal(2)
    np.testing.assert_allclose(cnn.conv3x3(x, w, b), cnn.conv3x3_loops(x, w, b), rtol=1e-12,
                               atol=1e-12)


def test_bf16_rounding_matches_torch():
    import torch

    rng = np.random.default_rng(1)
    vals = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.uniform(-20, 20, 1000),
                           [1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -0.0, 65504.0]])
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(vals), ref)
    assert cnn.bf16(1.0 + 2.0**-8) == 1.0  # tie to even
    assert cnn.bf16(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6


def test_loss_invariances_and_gradient():
    rng = np.random.default_rng(2)
    u = rng.standard_normal(50)
    p = rng.standard_normal(50)
    l0, g = cnn.loss_and_grad(p, u)
    assert cnn.loss_and_grad(-3.5 * p, u)[0] == pytest.approx(l0, rel=1e-13)
    assert cnn.loss_and_grad(2.0 * u, u)[0] == pytest.approx(0.0, abs=1e-14)
    assert abs(p @ g) <= 1e-12 * np.linalg.norm(p) * np.linalg.norm(g)  # 0-homogeneous
    h = 1e-6
    for i in range(0, 50, 7):
        e = np.zeros(50)
        e[i] = h
        fd = (cnn.loss_and_grad(p + e, u)[0] - cnn.loss_and_grad(p - e, u)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    params = cnn.init_params(4)
    # small biases so that ReLU boundaries are not degenerate
    params = [(w, 0.05 * rng.standard_normal(b.shape)) for w, b in params]
    x = rng.standard_normal((2, 6, 5))
    u = rng.standard_normal(6 * 6 * 5)

    def loss_of(vec):
        acts = cnn.forward(cnn.unflatten(vec), x, rounded=False)
        return cnn.loss_and_grad(cnn.output_vector(acts[-1]), u)[0]

    vec = cnn.flatten(params)
    acts = cnn.forward(params, x, rounded=False)
    _, gp = cnn.loss_and_grad(cnn.output_vector(acts[-1]), u)
    dout = np.transpose(gp.reshape(6, 5, 6), (2, 0, 1))  # back to (6, s, s) layout
    grads = cnn.backward(params, acts, dout, rounded=False)
    gvec = cnn.flatten(grads)
    idx = rng.choice(vec.size, 40, replace=False)
    # include every bias of the last layer and first-layer weights
    idx = np.concatenate([idx, np.arange(9 * 2 * 64 - 5, 9 * 2 * 64), [vec.size - 1]])
    h = 1e-5
    for i in idx:
        e = np.zeros_like(vec)
        e[i] = h
        fd = (loss_of(vec + e) - loss_of(vec - e)) / (2 * h)
        assert gvec[i] == pytest.approx(fd, rel=2e-4, abs=1e-9), i


def test_output_vector_layout():
    out = np.arange(6 * 2 * 3, dtype=float).reshape(6, 2, 3)
    v = cnn.output_vector(out)
    # node (i, j) = (1, 2), field f = 4 sits at 6*(1*3 + 2) + 4
    assert v[6 * (1 * 3 + 2) + 4] == out[4, 1, 2]


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    vec = rng.standard_normal(30)
    g = rng.standard_normal(30)
    new, m, v = cnn.adam_step(vec, g, np.zeros(30), np.zeros(30), 1, lr=1e-3)
    np.testing.assert_allclose(new, vec - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
