"""The learned-guess network on the GPU (BF16 MFMA kernels behind the C ABI)
against the NumPy oracle.

The oracle evaluates with the same BF16 rounding of weights, inputs,
activations and activation gradients, in FP64 sums; what remains is the
order of the FP32 accumulation and the odd BF16 rounding it flips (one BF16
ulp is 2^-8 relative).  Bar, norm-wise (max|a-b| / max|b|): 2e-3 for the
outputs, 1e-3 for the weight and bias gradients; Adam on FP32 to 1e-6.
"""
import sys

import numpy as np
import pytest

import oracle.nn as onn

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(P, nr, nz):
    # a context only provides the canvas shape and the stream here
    return P.Context(nr=nr, nz=nz, R=0.02, L=0.02, xi_a=2.0, dt=1e-11, eps=8.8541878128e-12,
                     mu=1.25663706212e-6)


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def _unflat(w):
    out, o = [], 0
    for ci, co in onn.LAYERS:
        W = w[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = w[o:o + co]
        o += co
        out.append((W, b))
    return out


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _case(seed, nimg, nr, nz):
    rng = np.random.default_rng(seed)
    params = onn.init_params(seed=seed)
    params = [(W, rng.standard_normal(W.shape[0]) * 0.05) for W, _ in params]
    w = _flat(params).astype(np.float32).astype(np.float64)
    x = onn.bf16(rng.standard_normal((nimg, 6, nr + 1, nz + 1)))
    return _unflat(w), w, x, rng


@pytest.mark.parametrize("shape", [(20, 40), (33, 70)])
def test_forward_matches_oracle(torch_cuda, shape):
    import paper_2212_08836_amd as P
    nr, nz = shape
    ctx = _ctx(P, nr, nz)
    assert ctx.nn_param_count() == sum(co * ci * 9 + co for ci, co in onn.LAYERS)
    params, w, x, _ = _case(1, 3, nr, nz)
    y = ctx.nn_forward(w, x).cpu().numpy().astype(np.float64)
    yo, _ = onn.forward(params, x, round_bf16=True)
    err = _rel(y, yo)
    _flush(f"  forward {shape}: rel err {err:.2e}")
    assert err < 2e-3


def test_gradient_matches_oracle(torch_cuda):
    import paper_2212_08836_amd as P
    nr, nz = 20, 40
    ctx = _ctx(P, nr, nz)
    params, w, x, rng = _case(2, 2, nr, nz)
    t = rng.standard_normal((2, 2, nr + 1, nz + 1)).astype(np.float32).astype(np.float64)
    dw, loss = ctx.nn_grad(w, x, t)
    dw = dw.cpu().numpy().astype(np.float64)
    yo, acts = onn.forward(params, x, round_bf16=True)
    mask = onn.masks(nr, nz)
    lo, dy = onn.mse(yo, t, mask)
    go = onn.backward(params, acts, dy, round_bf16=True)
    assert abs(loss - lo) <= 1e-3 * lo
    o = 0
    for k, (ci, co) in enumerate(onn.LAYERS):
        dW = dw[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        db = dw[o:o + co]
        o += co
        eW, eb = _rel(dW, go[k][0]), _rel(db, go[k][1])
        _flush(f"  layer {k}: dW rel err {eW:.2e}, db rel err {eb:.2e}")
        assert eW < 1e-3 and eb < 1e-3


def test_adam_matches_oracle(torch_cuda):
    import paper_2212_08836_amd as P
    torch = torch_cuda
    ctx = _ctx(P, 8, 8)
    n = ctx.nn_param_count()
    rng = np.random.default_rng(3)
    w0 = rng.standard_normal(n).astype(np.float32)
    wg = torch.tensor(w0, device="cuda")
    mg = torch.zeros(n, device="cuda")
    vg = torch.zeros(n, device="cuda")
    wo, mo, vo = w0.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        ctx.nn_adam(wg, mg, vg, torch.tensor(g, device="cuda"), 1e-3, step)
        wo, mo, vo = onn.adam_step(wo, mo, vo, g.astype(np.float64), step, lr=1e-3)
    torch.cuda.synchronize()
    assert np.abs(wg.cpu().numpy() - wo).max() < 1e-6
