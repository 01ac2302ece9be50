"""The learned initial guess inside the implicit step, trained on the GPU by
the library's own kernels on snapshots of the plain method (c2 physics).

What it must show:
  * the answer does not change: from a common state, a step with the
    learned guess and a step with the extrapolated guess converge to the
    same fields (to the Picard tolerance);
  * what the network gains: on held-out steps of a run it was not trained
    on, interleaving guessed and extrapolated steps, the first Picard
    residual (the distance of the guess from the converged field) and the
    iteration count, reported and compared.
"""
import sys

import numpy as np
import pytest

import ecpic_inputs as E

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


def _run(P, seed, pressure):
    w = E.workload("c2", seed=seed, pressure_pa=pressure)
    parts = E.make_particles(w)
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, parts, extra_cap=0.3)
    ctx.sort()
    ctx.set_mcc(w.mcc_params())
    return w, ctx


@pytest.fixture(scope="module")
def trained(torch_cuda):
    import paper_2212_08836_amd as P
    from paper_2212_08836_amd import nn_guess as G
    xs, ts = [], []
    for seed, pr in ((102, 5.0), (103, 2.0)):
        w, ctx = _run(P, seed, pr)
        for k in range(20):
            ctx.step(tol=w.tol, sort_every=4, stats=False)
        x, t = G.collect(ctx, 250, w.tol)
        xs.append(x)
        ts.append(t)
        ctx.close()
    x, t = np.concatenate(xs), np.concatenate(ts)
    norm = G.scales(x, t)
    w, ctx = _run(P, 2, 5.0)
    xd, td = G.to_device(ctx, x, t, norm)
    wts, losses = G.train(ctx, xd, td, steps=1200, batch=8, lr=1e-3, seed=1)
    _flush(f"  training loss {losses[0]:.3f} -> {np.mean(losses[-50:]):.3f} (scaled MSE)")
    assert np.mean(losses[-50:]) < 0.6 * losses[0]
    return w, ctx, wts, norm


def test_learned_guess_gain_on_held_out_steps(trained):
    w, ctx, wts, norm = trained
    ctx.nn_set_weights(wts, norm)
    for k in range(30):
        ctx.step(tol=w.tol, sort_every=4, stats=False)
    res = {False: [], True: []}
    for k in range(120):
        use = k % 2 == 1
        d = ctx.step(tol=w.tol, sort_every=4, use_nn=use)
        assert d["converged"] == 1 and d["residual"][d["iters"] - 1] <= w.tol
        assert d["used_nn"] == int(use)
        res[use].append((d["iters"], d["residual"][0], d["nn_fallback"]))
    plain, nn = np.array(res[False]), np.array(res[True])
    _flush(f"  extrapolated guess: iterations {plain[:, 0].mean():.3f}, first residual "
           f"mean {plain[:, 1].mean():.3e}")
    _flush(f"  learned guess:      iterations {nn[:, 0].mean():.3f}, first residual "
           f"mean {nn[:, 1].mean():.3e}, fallbacks {int(nn[:, 2].sum())}")
    # the gain: the learned guess is closer to the converged field
    assert nn[:, 1].mean() < 0.8 * plain[:, 1].mean()
    assert nn[:, 0].mean() <= plain[:, 0].mean() + 0.05


def test_learned_guess_does_not_change_the_answer(trained):
    import paper_2212_08836_amd as P
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    import test_gpu_mixed as T
    w, ctx, wts, norm = trained
    st = ctx.diagnostics()
    parts, fields = T._state_of(ctx, w)
    ref = E.make_particles(w)
    qmw = [(ref[k]["q"], ref[k]["m"], ref[k]["w"]) for k in range(2)]
    del ref
    caps = [int(len(p["r"]) * 1.2) + 256 for p in parts]
    a = T._fresh(P, w, "fp64", parts, fields, caps, qmw, st["t"], st["step"], w.mcc_params())
    b = T._fresh(P, w, "fp64", parts, fields, caps, qmw, st["t"], st["step"], w.mcc_params())
    b.nn_set_weights(wts, norm)
    da = a.step(tol=w.tol)
    db = b.step(tol=w.tol, use_nn=True)
    assert db["used_nn"] == 1 and da["converged"] == db["converged"] == 1
    fa, fb = a.get_fields(), b.get_fields()
    errs = [np.abs(x - y).max() / np.abs(y).max() for x, y in zip(fb, fa)]
    _flush(f"  learned vs extrapolated guess, same step: field rel diff {max(errs):.2e}, "
           f"first residual {db['residual'][0]:.2e} vs {da['residual'][0]:.2e}")
    # both are within the tolerance of the one converged answer
    assert max(errs) < 1e-8


def test_learned_guess_on_the_512x256_grid(torch_cuda):
    # the learned guess on the 512x256 grid (R = 0.25 m, 128 particles per
    # cell per species): trained there on snapshots of the plain method from
    # two other seeds and pressures, compared with the extrapolated guess on
    # held-out steps of a third run, at the same converged residual
    import paper_2212_08836_amd as P
    from paper_2212_08836_amd import nn_guess as G
    xs, ts = [], []
    for seed, pr in ((302, 5.0), (303, 2.0)):
        w = E.workload("c3", seed=seed, pressure_pa=pr)
        ctx = P.context_from_workload(w)
        P.load_workload_species(ctx, E.make_particles(w), extra_cap=0.3)
        ctx.sort()
        ctx.set_mcc(w.mcc_params())
        ctx.run(20, tol=w.tol, sort_every=8)
        x, t = G.collect(ctx, 130, w.tol, sort_every=8)
        xs.append(x)
        ts.append(t)
        ctx.close()
    x, t = np.concatenate(xs), np.concatenate(ts)
    norm = G.scales(x, t)
    w = E.workload("c3")
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, E.make_particles(w), extra_cap=0.3)
    ctx.sort()
    ctx.set_mcc(w.mcc_params())
    xd, td = G.to_device(ctx, x, t, norm)
    del x, t
    wts, losses = G.train(ctx, xd, td, steps=800, batch=8, lr=1e-3, seed=1)
    del xd, td
    _flush(f"  512x256: {len(xs[0]) + len(xs[1])} snapshots, training loss {losses[0]:.3f} -> "
           f"{np.mean(losses[-50:]):.3f}")
    ctx.nn_set_weights(wts, norm)
    ctx.run(20, tol=w.tol, sort_every=8)
    res = {False: [], True: []}
    for k in range(60):
        use = k % 2 == 1
        d = ctx.step(tol=w.tol, sort_every=8, use_nn=use)
        assert d["converged"] == 1 and d["residual"][d["iters"] - 1] <= w.tol
        res[use].append((d["iters"], d["residual"][0], d["nn_fallback"]))
    plain, nn = np.array(res[False]), np.array(res[True])
    _flush(f"  512x256 extrapolated guess: iterations {plain[:, 0].mean():.3f}, first residual "
           f"mean {plain[:, 1].mean():.3e}")
    _flush(f"  512x256 learned guess:      iterations {nn[:, 0].mean():.3f}, first residual "
           f"mean {nn[:, 1].mean():.3e}, fallbacks {int(nn[:, 2].sum())}")
    ctx.close()
    assert nn[:, 1].mean() < plain[:, 1].mean()
    assert nn[:, 0].mean() <= plain[:, 0].mean() + 0.05


def test_learned_guess_far_off_still_converges_to_the_answer(trained):
    # weights flipped in sign and scaled by 1e3: the guess is far off (first
    # residual ~1e7); Picard still contracts (no fallback needed) and ends at
    # the same converged answer, with the charge conserved
    import paper_2212_08836_amd as P
    a, b, w = _twin_states(P, trained)
    torch = pytest.importorskip("torch")
    _, _, wts, norm = trained
    b.nn_set_weights(torch.as_tensor(wts).clone() * -1e3, norm)
    da = a.step(tol=w.tol)
    db = b.step(tol=w.tol, use_nn=True, conservation=True)
    _flush(f"  corrupted network: fallback {db['nn_fallback']}, iterations {db['iters']} vs "
           f"{da['iters']}, residuals {['%.1e' % r for r in db['residual']]}")
    assert db["used_nn"] == 1 and db["converged"] == 1 and db["residual"][0] > 1e3
    _same_answer(a, b)
    assert db["continuity_max"] <= 1e-12 * db["q_max"]


@pytest.mark.parametrize("at", [1, 2, 3])
def test_learned_guess_fallback_restarts_cleanly(trained, at):
    # the fallback path, forced from the host at iteration `at`: the step
    # restarts from the extrapolated guess (or accepts an iteration already
    # enqueued ahead that converged), ends at the same answer, and no
    # speculative commit of the abandoned attempt leaves wall charge behind
    import paper_2212_08836_amd as P
    a, b, w = _twin_states(P, trained)
    _, _, wts, norm = trained
    b.nn_set_weights(wts, norm)
    b.set_option(P.ECPIC_OPT_NN_FORCE_FALLBACK, at)
    da = a.step(tol=w.tol)
    db = b.step(tol=w.tol, use_nn=True, conservation=True)
    _flush(f"  fallback forced at {at}: taken {db['nn_fallback']}, iterations {db['iters']} vs "
           f"{da['iters']}")
    assert db["used_nn"] == 1 and db["converged"] == 1
    # at k <= iters - 3 the restart is taken; at iters - 2 the iteration
    # enqueued ahead may already have converged (then it is accepted); at
    # iters - 1 the step converges before the check
    if at <= da["iters"] - 3:
        assert db["nn_fallback"] == 1
    if at == da["iters"] - 1:
        assert db["nn_fallback"] == 0
    _same_answer(a, b)
    assert db["continuity_max"] <= 1e-12 * db["q_max"]
    # two more steps: wall charge and fields stay with the plain context's
    for n in range(2):
        a.step(tol=w.tol)
        b.step(tol=w.tol, use_nn=True)
    _same_answer(a, b)


def _twin_states(P, trained):
    """Two FP64 contexts holding the trained context's current state."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    import test_gpu_mixed as T
    w, ctx, wts, norm = trained
    st = ctx.diagnostics()
    parts, fields = T._state_of(ctx, w)
    ref = E.make_particles(w)
    qmw = [(ref[k]["q"], ref[k]["m"], ref[k]["w"]) for k in range(2)]
    del ref
    caps = [int(len(p["r"]) * 1.2) + 256 for p in parts]
    a = T._fresh(P, w, "fp64", parts, fields, caps, qmw, st["t"], st["step"], w.mcc_params())
    b = T._fresh(P, w, "fp64", parts, fields, caps, qmw, st["t"], st["step"], w.mcc_params())
    return a, b, w


def _same_answer(a, b):
    fa, fb = a.get_fields(), b.get_fields()
    errs = [np.abs(x - y).max() / np.abs(y).max() for x, y in zip(fb, fa)]
    assert max(errs) < 1e-8, errs
    # wall charge totals (bottom, top, side)
    qa, qb = a.node_charge(), b.node_charge()
    for x, y in zip(qa[1:], qb[1:]):
        assert np.abs(x - y).max() <= 1e-6 * max(np.abs(y).max(), 1e-300)
