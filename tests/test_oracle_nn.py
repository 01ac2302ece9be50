"""Pins of the NumPy oracle of the learned guess (CPU only): the convolution
against SciPy's 2-D correlation, every gradient against central finite
differences, Adam against its defining properties, bfloat16 rounding against
torch's conversion and hand-worked ties."""
import numpy as np
import pytest

import oracle.nn as nn


def test_conv_matches_scipy_correlate():
    from scipy.signal import correlate2d
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 7, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = nn.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], W[o, c], mode="same") for c in range(3))
            assert np.allclose(y[n, o], ref, rtol=0, atol=1e-12)


def _fd(f, a, idx, h=1e-6):
    a0 = a[idx]
    a[idx] = a0 + h
    fp = f()
    a[idx] = a0 - h
    fm = f()
    a[idx] = a0
    return (fp - fm) / (2 * h)


def test_input_and_weight_grads_by_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 6, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    R = rng.standard_normal((2, 4, 6, 5))
    f = lambda: (nn.conv3x3(x, W, b) * R).sum()
    dx = nn.conv3x3_input_grad(R, W)
    dW, db = nn.conv3x3_weight_grad(x, R)
    for _ in range(12):
        i = tuple(rng.integers(0, s) for s in x.shape)
        assert abs(_fd(f, x, i) - dx[i]) <= 1e-7 * max(1.0, abs(dx[i]))
        j = tuple(rng.integers(0, s) for s in W.shape)
        assert abs(_fd(f, W, j) - dW[j]) <= 1e-7 * max(1.0, abs(dW[j]))
    for o in range(4):
        assert abs(_fd(f, b, (o,)) - db[o]) <= 1e-7 * max(1.0, abs(db[o]))


def test_network_backward_by_finite_differences():
    rng = np.random.default_rng(3)
    params = nn.init_params(seed=4)
    # nonzero biases so that ReLU kinks are away from the probes
    params = [(W, rng.standard_normal(W.shape[0]) * 0.1) for W, _ in params]
    x = rng.standard_normal((2, 6, 6, 5))
    t = rng.standard_normal((2, 2, 6, 5))
    mask = np.ones((2, 6, 5))
    mask[0, :, 0] = 0.0

    def loss():
        y, _ = nn.forward(params, x)
        return nn.mse(y, t, mask)[0]

    y, acts = nn.forward(params, x)
    _, dy = nn.mse(y, t, mask)
    grads = nn.backward(params, acts, dy)
    for k, (W, b) in enumerate(params):
        for _ in range(6):
            j = tuple(rng.integers(0, s) for s in W.shape)
            g = grads[k][0][j]
            assert abs(_fd(loss, W, j, 1e-5) - g) <= 1e-6 * max(1e-3, abs(g)), (k, j)
        o = (int(rng.integers(0, b.shape[0])),)
        g = grads[k][1][o]
        assert abs(_fd(loss, b, o, 1e-5) - g) <= 1e-6 * max(1e-3, abs(g)), (k, "bias")


def test_adam_first_step_and_convergence():
    rng = np.random.default_rng(5)
    g = rng.standard_normal(50)
    w = np.zeros(50)
    w1, m, v = nn.adam_step(w, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    # bias-corrected first step: lr * g / (|g| + eps)
    assert np.allclose(w1, -1e-3 * np.sign(g), rtol=1e-6, atol=0)
    target = rng.standard_normal(50)
    w, m, v = np.zeros(50), np.zeros(50), np.zeros(50)
    for t in range(1, 4001):
        w, m, v = nn.adam_step(w, m, v, w - target, t, lr=1e-2)
    assert np.abs(w - target).max() < 1e-3


def test_bf16_rounding():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8)]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nn.bf16(x), ref)
    # ties to even, worked by hand
    assert nn.bf16(1.0 + 2.0 ** -8) == 1.0
    assert nn.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_canvas_and_masks():
    nr, nz = 4, 3
    ur = np.arange(nr * (nz + 1), dtype=float) + 1
    uz = -np.arange((nr + 1) * nz, dtype=float) - 1
    h = np.arange(nr * nz, dtype=float) + 100
    c = nn.canvas(ur, uz, h, nr, nz)
    assert c[0, nr, :].sum() == 0 and c[1, :, nz].sum() == 0
    assert c[0, 2, 3] == ur.reshape(nr, nz + 1)[2, 3]
    assert c[1, 4, 1] == uz.reshape(nr + 1, nz)[4, 1]
    assert c[2, 1, 2] == h.reshape(nr, nz)[1, 2]
    m = nn.masks(nr, nz)
    assert m[0].sum() == nr * (nz - 1) and m[1].sum() == nr * nz
