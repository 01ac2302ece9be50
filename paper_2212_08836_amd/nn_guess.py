"""Training driver of the learned Picard initial guess.

The network (see ecpic_nn_* in include/ecpic.h) maps the field state at t^n
to the correction of the extrapolated guess 2u^n - u^{n-1} of u^{n+1}.  The
training pairs come from the plain method itself: a context steps with the
extrapolated guess to the Picard tolerance, and each converged step gives one
(input canvas, target correction) pair.  Forward, backward and Adam run in the
library's kernels; this module only gathers the snapshots, picks the channel
scales and loops.
"""
from __future__ import annotations

import numpy as np

N_IN, N_OUT = 6, 2


def canvas_channels(ur, uz, h, ur_p, uz_p, h_p, nr, nz):
    """The six unscaled input channels on the (nr+1) x (nz+1) canvas:
    u_r, u_z, h at t^n and their change since t^{n-1}, each at its own
    index (i, j), zero elsewhere."""
    c = np.zeros((N_IN, nr + 1, nz + 1))
    ur, uz, h = (np.asarray(a).reshape(s) for a, s in
                 ((ur, (nr, nz + 1)), (uz, (nr + 1, nz)), (h, (nr, nz))))
    ur_p, uz_p, h_p = (np.asarray(a).reshape(s) for a, s in
                       ((ur_p, (nr, nz + 1)), (uz_p, (nr + 1, nz)), (h_p, (nr, nz))))
    c[0, :nr, :] = ur
    c[1, :, :nz] = uz
    c[2, :nr, :nz] = h
    c[3, :nr, :] = ur - ur_p
    c[4, :, :nz] = uz - uz_p
    c[5, :nr, :nz] = h - h_p
    return c


def target_channels(ur1, uz1, ur, uz, ur_p, uz_p, nr, nz):
    """u^{n+1} - (2u^n - u^{n-1}) for u_r and u_z on the canvas."""
    t = np.zeros((N_OUT, nr + 1, nz + 1))
    d_r = np.asarray(ur1) - (2.0 * np.asarray(ur) - np.asarray(ur_p))
    d_z = np.asarray(uz1) - (2.0 * np.asarray(uz) - np.asarray(uz_p))
    t[0, :nr, :] = d_r.reshape(nr, nz + 1)
    t[1, :, :nz] = d_z.reshape(nr + 1, nz)
    return t


def collect(ctx, steps, tol, sort_every=4, skip=5):
    """Step `ctx` (plain guess) and return the unscaled inputs [S][6][H][W]
    and targets [S][2][H][W] of the steps after the first `skip`."""
    nr, nz = ctx.nr, ctx.nz
    xs, ts = [], []
    prev = ctx.get_fields()
    cur = prev
    for k in range(steps):
        ctx.step(tol=tol, sort_every=sort_every, stats=False)
        nxt = ctx.get_fields()
        if k >= skip:
            xs.append(canvas_channels(cur[0], cur[1], cur[2], prev[0], prev[1], prev[2], nr, nz))
            ts.append(target_channels(nxt[0], nxt[1], cur[0], cur[1], prev[0], prev[1], nr, nz))
        prev, cur = cur, nxt
    return np.stack(xs), np.stack(ts)


def scales(x, t):
    """Per-channel RMS of the training inputs and targets (floored)."""
    s_in = np.sqrt((x ** 2).mean(axis=(0, 2, 3)))
    s_out = np.sqrt((t ** 2).mean(axis=(0, 2, 3)))
    s_in = np.where(s_in > 0, s_in, 1.0)
    s_out = np.where(s_out > 0, s_out, 1.0)
    return np.concatenate([s_in, s_out]).astype(np.float32)


def init_weights(n_params_expected, seed=0):
    """He-normal FP32 weights in the canonical layout, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in ((6, 32), (32, 32), (32, 32), (32, 2)):
        parts.append(rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)))
        parts.append(np.zeros(co))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == n_params_expected
    return w


def to_device(ctx, x, t, norm):
    """Scaled BF16 inputs and FP32 targets on the device."""
    torch = ctx.torch
    s_in = norm[:N_IN].astype(np.float64)[None, :, None, None]
    s_out = norm[N_IN:].astype(np.float64)[None, :, None, None]
    xd = torch.tensor((x / s_in).astype(np.float32), device=ctx.device).to(torch.bfloat16)
    td = torch.tensor((t / s_out).astype(np.float32), device=ctx.device)
    return xd, td


def train(ctx, xd, td, steps=400, batch=8, lr=1e-3, seed=0, w=None, progress=None):
    """Adam on the mean squared error; returns the FP32 weights (device) and
    the loss history.  progress(step, loss) is called every 100 steps."""
    torch = ctx.torch
    n = ctx.nn_param_count()
    if w is None:
        w = torch.tensor(init_weights(n, seed), device=ctx.device)
    m = torch.zeros(n, device=ctx.device)
    v = torch.zeros(n, device=ctx.device)
    rng = np.random.default_rng(seed)
    losses = []
    S = xd.shape[0]
    for it in range(1, steps + 1):
        idx = torch.tensor(rng.choice(S, size=min(batch, S), replace=False), device=ctx.device)
        dw, loss = ctx.nn_grad(w, xd.index_select(0, idx).contiguous(),
                               td.index_select(0, idx).contiguous())
        ctx.nn_adam(w, m, v, dw, lr, it)
        losses.append(loss)
        if progress is not None and it % 100 == 0:
            progress(it, loss)
    torch.cuda.synchronize()
    return w, losses
