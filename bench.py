"""Benchmark of the implicit EM PIC/MCC hot path on one MI355X.

Workload: the 256 x 128 VHF CCP slab (R = 0.15 m, L = 3 cm, 100 MHz / 200 V
drive on the bottom electrode, J0(2.405 r/R) sin(pi z/L) density of 1e16
m^-3, 64 macro-particles per cell per species = 4,194,304 particles,
null-collision MCC in 5 Pa argon, dt = 1e-11 s, Picard tolerance 1e-10),
plain FP64 path.  A step is one implicit step: guess, Picard iterations of
push+deposit and field solve, commit with absorption and MCC, and the
counting sort every 16 steps.  Synthetic seeded inputs, resident in HBM
before the timed region.

Prints one JSON line.  `value` = particle-pushes per second counted over the
Picard iterations (N_alive x iterations summed over the timed steps, divided
by the wall time of the whole steps).  `mixed_nn` gives the same workload in
the FP32-push form with the learned initial guess (trained beforehand, outside
the timed region, on snapshots of the plain method from other seeds), its
seconds per step and speedup over the plain FP64 path.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM traffic of the dominant kernel, taken with rocprofv3 --pmc (FETCH_SIZE,
# then WRITE_SIZE) and scaled by what the same counters read for a streaming
# copy of known size (the --calibrate-copy mode below).  Reported only while
# the kernel sources hash to what they were when the counters were taken.
WORKLOADS = {
    "c2": "VHF CCP slab 256x128 (R 0.15 m, L 3 cm), 4.19M particles, 100 MHz 200 V, MCC 5 Pa",
    "c3": "VHF CCP slab 512x256 (R 0.25 m, L 3 cm), 33.5M particles, 100 MHz 200 V, MCC 5 Pa",
    "c5": "dual-frequency CCP 1024x512 (R 0.3 m, L 3 cm), 268M particles, 60 + 13.56 MHz "
          "200 V each, MCC 5 Pa",
}
EVENT_EVERY = 8  # timed-region launches of the dominant kernel carrying events
RUN_CHUNK = 50   # steps per library call in the timed region
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_push_fast_c2_{precision}_traffic.txt")
PUSH_SOURCES = ("paper_2212_08836_amd/csrc/ecpic_push.hip",
                "paper_2212_08836_amd/csrc/ecpic_internal.h")


def push_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PUSH_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(precision):
    """Bytes per launch of the fast push from the committed counter summary,
    or None when absent or taken on other kernel sources."""
    path = TRAFFIC_FILE.format(precision=precision)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != push_source_hash() or vals.get("precision") != precision:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def mixed_nn_leg(E, P, w, parts, steps, warmup, sort_every, plain_ms, self_train=False):
    """The FP32 push + learned-guess form on the same workload.  The network
    is trained first (outside the timed region) by the library's kernels: on
    snapshots of the plain FP64 method from two other seeds/pressures, or
    (self_train, for the larger grids) on snapshots of the mixed run's own
    first steps with the extrapolated guess."""
    import torch
    from paper_2212_08836_amd import nn_guess as G
    t0 = time.perf_counter()
    ctx = P.context_from_workload(w, precision="mixed")
    P.load_workload_species(ctx, parts, extra_cap=0.25)
    ctx.sort()
    ctx.set_mcc(w.mcc_params())
    if self_train:
        ctx.run(20, tol=w.tol, sort_every=sort_every)
        x, t = G.collect(ctx, 125, w.tol, sort_every=sort_every)
        adam_steps = 400
    else:
        xs, ts = [], []
        for seed, pr in ((102, 5.0), (103, 2.0)):
            wt = E.workload(w.name, seed=seed, pressure_pa=pr)
            c = P.context_from_workload(wt)
            P.load_workload_species(c, E.make_particles(wt), extra_cap=0.3)
            c.sort()
            c.set_mcc(wt.mcc_params())
            c.run(20, tol=wt.tol, sort_every=sort_every)
            x, t = G.collect(c, 250, wt.tol, sort_every=sort_every)
            xs.append(x)
            ts.append(t)
            c.close()
        x, t = np.concatenate(xs), np.concatenate(ts)
        del xs, ts
        adam_steps = 1200
    n_snap = int(x.shape[0])
    norm = G.scales(x, t)
    print(f"# mixed + learned guess: {n_snap} snapshots collected", file=sys.stderr, flush=True)
    xd, td = G.to_device(ctx, x, t, norm)
    del x, t
    wts, losses = G.train(ctx, xd, td, steps=adam_steps, batch=8, lr=1e-3, seed=1)
    del xd, td
    ctx.nn_set_weights(wts, norm)
    t_train = time.perf_counter() - t0
    print(f"# mixed + learned guess: trained in {t_train:.1f} s, loss {losses[0]:.3f} -> "
          f"{np.mean(losses[-50:]):.3f}", file=sys.stderr, flush=True)
    ctx.run(warmup, tol=w.tol, sort_every=sort_every, use_nn=True)
    torch.cuda.synchronize()
    # counts only (the first launch of a kind is the only one timed)
    ctx.set_profiling(True, kinds=("push", "push_commit"), every=1 << 30)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k = 0
    while k < steps:
        n = min(RUN_CHUNK, steps - k)
        ctx.run(n, tol=w.tol, sort_every=sort_every, use_nn=True)
        k += n
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    prof = ctx.profile()
    ctx.set_profiling(False)
    # first residual and fallbacks over a few steps with statistics
    r0, fb = [], 0
    for k in range(20):
        d = ctx.step(tol=w.tol, sort_every=sort_every, use_nn=True)
        r0.append(d["residual"][0])
        fb += d["nn_fallback"]
    ctx.close()
    ms = 1e3 * el / steps
    return {"ms_per_step": ms, "s_per_step": el / steps,
            "particle_pushes_per_s": (prof["push"]["call_particles"] +
                                      prof["push_commit"]["call_particles"]) / el,
            "picard_iterations_per_step": (prof["push"]["calls"] +
                                           prof["push_commit"]["calls"]) / steps,
            "first_residual_mean": float(np.mean(r0)), "nn_fallbacks": fb,
            "speedup_vs_plain": plain_ms / ms,
            "train": {"snapshots": n_snap, "adam_steps": len(losses),
                      "loss_first": losses[0], "loss_last50": float(np.mean(losses[-50:])),
                      "seconds": t_train}}


def calibrate_copy(mib):
    """A streaming copy of known size (negation of a float64 buffer into a
    second one: `mib` MiB read and written per launch), run a few times so
    that rocprofv3 --pmc can relate FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "neg float64", "bytes_read": n * 8, "bytes_written": n * 8,
                      "launches": 5}), flush=True)


def cpu_baseline(w, parts, mcc, steps=3):
    """The FP64 oracle, single-threaded, on the same workload: the full
    particle set on the full grid, three implicit steps from the initial load
    (about 15 s)."""
    import oracle as og
    g = og.grid_from_workload(w)
    sp = og.species_from_workload(g, parts, extra_cap=0.05)
    st = og.State(g)
    t0 = time.perf_counter()
    pushes = 0
    iters = []
    for _ in range(steps):
        n_alive = sum(s.n for s in sp)
        d = g.step(st, sp, mcc=mcc, tol=w.tol)
        pushes += n_alive * d["iters"]
        iters.append(d["iters"])
    dt = time.perf_counter() - t0
    return {"value": pushes / dt, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
            "s_per_step": dt / steps,
            "sample": f"{steps} implicit step(s) of the full workload "
                      f"({sum(len(p['r']) for p in parts)} particles, 256x128 grid, MCC), "
                      f"Picard iterations {iters}, single-threaded C oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS),
                    help="c2 is the measured configuration; the larger ones are reported "
                         "on request (no oracle baseline, network trained on the run itself)")
    ap.add_argument("--sort-every", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-nn", action="store_true",
                    help="skip the FP32 push + learned-guess comparison")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run the streaming copy used to scale the HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import ecpic_inputs as E
    import paper_2212_08836_amd as P

    torch.cuda.set_device(0)
    w = E.workload(args.workload)
    print(f"# generating the {args.workload} particles", file=sys.stderr, flush=True)
    parts = E.make_particles(w)
    n0 = sum(len(p["r"]) for p in parts)
    ctx = P.context_from_workload(w, precision=args.precision)
    P.load_workload_species(ctx, parts, extra_cap=0.25)
    ctx.sort()
    mcc = w.mcc_params()
    ctx.set_mcc(mcc)
    print(f"# bench: {args.workload} {w.nr}x{w.nz}, {n0} particles, {args.precision}, "
          f"warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)
    ctx.run(args.warmup, tol=w.tol, sort_every=args.sort_every)
    torch.cuda.synchronize()
    # in the timed region only the in-cell passes are counted (a committing
    # iteration's pass pushes too), and only every 8th launch of each carries
    # timing events: an event record stalls the stream for a few
    # microseconds, so timing every launch would stretch the step
    ctx.set_profiling(True, kinds=("push", "push_commit"), every=EVENT_EVERY)
    torch.cuda.synchronize()
    # the steps run inside the library (ecpic_run), in chunks so that
    # progress can be reported
    t0 = time.perf_counter()
    last_print = t0
    k = 0
    while k < args.steps:
        n = min(RUN_CHUNK, args.steps - k)
        ctx.run(n, tol=w.tol, sort_every=args.sort_every)
        k += n
        now = time.perf_counter()
        if now - last_print > 20:
            print(f"# step {k}", file=sys.stderr, flush=True)
            last_print = now
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile()
    # per-kind kernel times from a short untimed run with every kind timed
    ctx.set_profiling(True)
    for k in range(min(args.steps, 2 * args.sort_every if args.sort_every > 0 else 8)):
        ctx.step(tol=w.tol, sort_every=args.sort_every, stats=False)
    prof_all = ctx.profile()
    ctx.set_profiling(False)
    elapsed = t1 - t0
    # Picard iterations: one in-cell (fast) push launch per iteration over
    # the particles of both species; the face crossers are redone in the
    # slow pass that follows it
    push = prof["push"]
    n_push_passes = push["calls"] + prof["push_commit"]["calls"]
    pushes = push["call_particles"] + prof["push_commit"]["call_particles"]
    value = pushes / elapsed
    avg_launch_ms = push["ms"] / push["launches"]
    bytes_per_launch = push["bytes"] / push["launches"]
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    diag = ctx.diagnostics()
    out = {
        "metric": "particle-pushes/s per Picard iteration (and s per implicit step)",
        "value": value,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "s_per_step": elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "particles": n0, "grid": [w.nr, w.nz], "dt": w.dt, "tol": w.tol,
                   "precision": args.precision, "sort_every": args.sort_every,
                   "parallelism": "single GPU"},
        "picard_iterations_per_step": n_push_passes / args.steps,
        "particles_alive_end": diag["n_alive"][:2],
        "kernel_ms": {k: (v["ms"] / v["launches"] if v["launches"] else None)
                      for k, v in prof_all.items()},
        "roofline": {"bound": "hbm", "kernel": ("k_push_fast<double, false, true>" if args.precision == "fp64" else
                                "k_push_fast<float, false, true>") + " (Picard iteration pass, both species)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": committed_traffic(args.precision) if args.workload == "c2" else None,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_launch_ms},
    }
    # first Picard residual of the plain (extrapolated) guess, for comparison
    r0 = []
    for k in range(20):
        r0.append(ctx.step(tol=w.tol, sort_every=args.sort_every)["residual"][0])
    out["first_residual_mean"] = float(np.mean(r0))
    if not args.no_nn and args.precision == "fp64":
        print("# mixed precision + learned guess", file=sys.stderr, flush=True)
        out["mixed_nn"] = mixed_nn_leg(E, P, w, parts, args.steps, args.warmup, args.sort_every,
                                       out["ms_per_step"], self_train=args.workload != "c2")
    if not args.no_cpu and args.workload == "c2":
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, parts, mcc)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
