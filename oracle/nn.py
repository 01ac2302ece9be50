"""Plain NumPy FP64 oracle of the learned Picard initial guess.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
timing may use this module.  It shares nothing with the HIP kernels.

The network is not part of the paper; it is the learned initial guess of the
implicit iteration of Sec. 2.1 (Picard on the coupled field/orbit system):
a small convolutional net maps the field state at t^n to a correction of the
extrapolated guess 2u^n - u^{n-1} of u^{n+1}.

Definitions (written out plainly):
  * layer l: y = conv3x3(x, W_l) + b_l, zero padding of one cell, stride 1,
    cross-correlation: y[n,o,i,j] = b[o] + sum_{c,p,q} W[o,c,p,q] x[n,c,i+p-1,j+q-1];
  * ReLU after every layer but the last;
  * loss: mean of (y - t)^2 over the entries where the mask is 1;
  * Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
Optionally every weight, input, activation and activation gradient is
rounded to bfloat16 (round to nearest even from float32), as the GPU stores
them; biases stay unrounded (FP32 on the GPU) and the sums are FP64 here.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((6, 32), (32, 32), (32, 32), (32, 2))


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    # NaN/inf stay as they are (not produced by the tests)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def init_params(seed=0, layers=LAYERS, scale=1.0):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for ci, co in layers:
        std = scale * np.sqrt(2.0 / (ci * 9))
        params.append((rng.standard_normal((co, ci, 3, 3)) * std, np.zeros(co)))
    return params


def conv3x3(x, W, b):
    """y[n,o,i,j] = b[o] + sum_{c,p,q} W[o,c,p,q] x[n,c,i+p-1,j+q-1] (zero pad)."""
    n, c, h, w = x.shape
    xp = np.zeros((n, c, h + 2, w + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((n, W.shape[0], h, w)) + b[None, :, None, None]
    for p in range(3):
        for q in range(3):
            y += np.einsum("oc,ncij->noij", W[:, :, p, q], xp[:, :, p:p + h, q:q + w])
    return y


def conv3x3_input_grad(dy, W):
    """dx[n,c,i,j] = sum_{o,p,q} W[o,c,p,q] dy[n,o,i-p+1,j-q+1] (zero outside)."""
    n, o, h, w = dy.shape
    dyp = np.zeros((n, o, h + 2, w + 2))
    dyp[:, :, 1:-1, 1:-1] = dy
    dx = np.zeros((n, W.shape[1], h, w))
    for p in range(3):
        for q in range(3):
            # dy at (i - p + 1, j - q + 1) sits at padded index (i - p + 2, j - q + 2)
            dx += np.einsum("oc,noij->ncij", W[:, :, p, q],
                            dyp[:, :, 2 - p:2 - p + h, 2 - q:2 - q + w])
    return dx


def conv3x3_weight_grad(x, dy):
    """dW[o,c,p,q] = sum_{n,i,j} dy[n,o,i,j] x[n,c,i+p-1,j+q-1]; db[o] = sum dy."""
    n, c, h, w = x.shape
    xp = np.zeros((n, c, h + 2, w + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dW = np.zeros((dy.shape[1], c, 3, 3))
    for p in range(3):
        for q in range(3):
            dW[:, :, p, q] = np.einsum("noij,ncij->oc", dy, xp[:, :, p:p + h, q:q + w])
    return dW, dy.sum(axis=(0, 2, 3))


def forward(params, x, round_bf16=False):
    """Returns the output and the per-layer inputs (for the backward pass)."""
    r = bf16 if round_bf16 else (lambda a: a)
    acts = []
    a = r(x)
    for k, (W, b) in enumerate(params):
        acts.append(a)
        y = conv3x3(a, r(W), b)
        if k + 1 < len(params):
            a = r(np.maximum(y, 0.0))
        else:
            a = y
    return a, acts


def mse(y, t, mask):
    cnt = mask.sum() * y.shape[0]
    d = (y - t) * mask
    return (d * d).sum() / cnt, 2.0 * d / cnt


def backward(params, acts, dy, round_bf16=False):
    """Gradients of the loss with respect to every weight and bias, given
    dL/dy of the last layer.  ReLU masks come from the stored layer inputs."""
    r = bf16 if round_bf16 else (lambda a: a)
    grads = [None] * len(params)
    g = r(dy)
    for k in range(len(params) - 1, -1, -1):
        W, b = params[k]
        dW, db = conv3x3_weight_grad(acts[k], g)
        grads[k] = (dW, db)
        if k > 0:
            dx = conv3x3_input_grad(g, r(W))
            g = r(dx * (acts[k] > 0.0))
    return grads


def adam_step(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place of copies; t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def canvas(ur, uz, h, nr, nz):
    """Index-aligned packing of the staggered arrays onto (nr+1) x (nz+1)."""
    out = np.zeros((3, nr + 1, nz + 1))
    out[0, :nr, :] = np.asarray(ur).reshape(nr, nz + 1)
    out[1, :, :nz] = np.asarray(uz).reshape(nr + 1, nz)
    out[2, :nr, :nz] = np.asarray(h).reshape(nr, nz)
    return out


def masks(nr, nz):
    """Output positions that are unknowns of the guess: interior r-edges
    (i < nr, 0 < j < nz) and z-edges off the PEC wall (i < nr, j < nz)."""
    m = np.zeros((2, nr + 1, nz + 1))
    m[0, :nr, 1:nz] = 1.0
    m[1, :nr, :nz] = 1.0
    return m
