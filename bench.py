"""Benchmark of the implicit EM PIC/MCC hot path on one MI355X.

Default workload: the largest single-GPU case, the dual-frequency CCP on a
1024 x 512 grid (R = 0.3 m, L = 3 cm, 60 MHz + 13.56 MHz at 200 V each on
the bottom electrode, J0(2.405 r/R) sin(pi z/L) density of 1e16 m^-3, 256
macro-particles per cell per species = 268,435,456 particles, null-collision
MCC in 5 Pa argon, dt = 1e-11 s, Picard tolerance 1e-10).  The particles are
drawn on the GPU by the seeded input generator and are resident in HBM, in
one torch-allocated region bound to the library, before the timed region.

A step is one implicit step: guess, Picard iterations of push+deposit and
field solve, commit with wall absorption and MCC, and the counting sort by
cell once per sort period.  The timed window starts right after a sort and
holds a whole number of sort periods (the period is the largest divisor of
the step count not above 32).

Prints one JSON line.  `value` = particle-pushes per second counted over the
Picard iterations (particles x iterations summed over the timed steps,
divided by the wall time of the whole steps), plain FP64 path.  `legs`
gives the same workload as FP32 push (mixed precision), FP64 with the
learned initial guess, and FP32 push with the learned guess: seconds per
step, iterations, and the speedup over the plain path.  The network is
trained beforehand, outside the timed region, on snapshots of the plain
method from two other seeds and pressures (held out from the timed run).
`roofline` is that of push+deposit (the in-cell pass and the slow pass of
the face crossers of one Picard iteration, both species): algorithmic bytes
(the particle state read once, 40 B per particle in FP64) over the summed
mean durations of the two launches, from HIP events on the library's stream.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    "c2": "VHF CCP slab 256x128 (R 0.15 m, L 3 cm), 4.19M particles, 100 MHz 200 V, MCC 5 Pa",
    "c3": "VHF CCP slab 512x256 (R 0.25 m, L 3 cm), 33.5M particles, 100 MHz 200 V, MCC 5 Pa",
    "c5": "dual-frequency CCP 1024x512 (R 0.3 m, L 3 cm), 268M particles, 60 + 13.56 MHz "
          "200 V each, MCC 5 Pa",
}
EVENT_EVERY = 8  # timed-region launches of a kind carrying events
RUN_CHUNK = 16   # steps per library call in the timed region
# HBM traffic of push+deposit, taken with rocprofv3 --pmc (FETCH_SIZE, then
# WRITE_SIZE) and scaled by what the same counters read for a streaming copy
# of known size (the --calibrate-copy mode).  Reported only while the kernel
# sources hash to what they were when the counters were taken.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "push_deposit_{workload}_{precision}_traffic.txt")
PUSH_SOURCES = ("paper_2212_08836_amd/csrc/ecpic_push.hip",
                "paper_2212_08836_amd/csrc/ecpic_internal.h")


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def push_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PUSH_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(workload, precision):
    """HBM bytes per push+deposit pass from the committed counter summary,
    or None when absent or taken on other kernel sources."""
    path = TRAFFIC_FILE.format(workload=workload, precision=precision)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != push_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_pass"])
    except (KeyError, ValueError):
        return None


# steps between counting sorts, measured per workload (the sorted order
# decays faster where the cells are small against a step's travel)
SORT_EVERY = {"c5": 16}
# the ions (0.026 eV) hardly move between sorts: the steps' sorts include
# them at every ION_SORT_STRIDE-th one
ION_SORT_STRIDE = {"c5": 4}
SORT_STRIDES = (1, 1)


def sort_period(steps, cap=32):
    """The largest divisor of `steps` not above cap."""
    for p in range(min(cap, steps), 0, -1):
        if steps % p == 0:
            return p
    return 1


def particles(E, w, device_gen):
    if device_gen:
        return E.make_particles_device(w, device="cuda")
    return E.make_particles(w)


def new_context(E, P, w, parts, precision, model="em", krylov=0, **over):
    """A context whose device memory is one torch tensor (bound workspace);
    krylov > 0 reserves that many JFNK Krylov vectors in it; over: grid
    settings in place of the workload's (port, blocking capacitor)."""
    ctx = P.context_from_workload(w, precision=precision, model=model, **over)
    if krylov:
        ctx.set_option(P.ECPIC_OPT_JFNK_KRYLOV, krylov)
    P.load_workload_species(ctx, parts, extra_cap=0.25, workspace=True, sort_strides=SORT_STRIDES)
    ctx.sort()
    ctx.set_mcc(w.mcc_params())
    return ctx


def timed_run(ctx, w, steps, warmup, period, use_nn=False, kinds=("push", "push_slow",
                                                                  "push_commit"), **solver):
    """Warm-up, alignment to a sort boundary, then `steps` timed steps
    (solver: ecpic_step options such as solver="jfnk", krylov, eta).
    Returns (elapsed seconds, profile of the timed region)."""
    import torch
    ctx.run(warmup, tol=w.tol, sort_every=period, use_nn=use_nn, **solver)
    step = ctx.diagnostics()["step"]
    if step % period:
        ctx.run(period - step % period, tol=w.tol, sort_every=period, use_nn=use_nn, **solver)
    torch.cuda.synchronize()
    ctx.set_profiling(True, kinds=kinds, every=EVENT_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    k = 0
    while k < steps:
        n = min(RUN_CHUNK, steps - k)
        ctx.run(n, tol=w.tol, sort_every=period, use_nn=use_nn, **solver)
        k += n
        if time.perf_counter() - last > 20:
            log(f"step {k}")
            last = time.perf_counter()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile()
    ctx.set_profiling(False)
    return elapsed, prof


def pushes_and_iters(prof, steps):
    passes = prof["push"]["calls"] + prof["push_commit"]["calls"]
    pushes = prof["push"]["call_particles"] + prof["push_commit"]["call_particles"]
    return pushes, passes / steps


def first_residuals(ctx, w, period, use_nn, n=8):
    r0, fb, iters = [], 0, []
    for _ in range(n):
        d = ctx.step(tol=w.tol, sort_every=period, use_nn=use_nn)
        r0.append(d["residual"][0])
        fb += d["nn_fallback"]
        iters.append(d["iters"])
    return float(np.mean(r0)), fb, float(np.mean(iters))


def train_network(E, P, G, w, period, device_gen, snapshots=64, adam_steps=600):
    """The learned guess, trained by the library's kernels on snapshots of
    the plain FP64 method from two held-out seeds and pressures."""
    t0 = time.perf_counter()
    xs, ts = [], []
    ctx = None
    for seed, pr in ((w.seed + 100, 5.0), (w.seed + 101, 2.0)):
        wt = E.workload(w.name, seed=seed, pressure_pa=pr)
        c = new_context(E, P, wt, particles(E, wt, device_gen), "fp64")
        c.run(16, tol=wt.tol, sort_every=period)
        x, t = G.collect(c, snapshots, wt.tol, sort_every=period)
        log(f"learned guess: {len(x)} snapshots of seed {seed} at {pr} Pa")
        xs.append(x)
        ts.append(t)
        if ctx is None:
            ctx = c
        else:
            c.close()
    x, t = np.concatenate(xs), np.concatenate(ts)
    del xs, ts
    norm = G.scales(x, t)
    xd, td = G.to_device(ctx, x, t, norm)
    n_snap = int(x.shape[0])
    del x, t
    wts, losses = G.train(ctx, xd, td, steps=adam_steps, batch=8, lr=1e-3, seed=1,
                          progress=lambda it, loss: log(f"adam step {it}: loss {loss:.3f}"))
    wts = wts.clone()
    del xd, td
    ctx.close()
    secs = time.perf_counter() - t0
    log(f"learned guess: {n_snap} held-out snapshots, loss {losses[0]:.3f} -> "
        f"{np.mean(losses[-50:]):.3f}, {secs:.0f} s")
    return wts, norm, {"snapshots": n_snap, "adam_steps": len(losses), "loss_first": losses[0],
                       "loss_last50": float(np.mean(losses[-50:])), "seconds": secs,
                       "held_out_seeds": [w.seed + 100, w.seed + 101],
                       "pressures_pa": [5.0, 2.0]}


def leg(E, P, w, parts_fn, precision, use_nn, steps, warmup, period, plain_ms, nn=None):
    ctx = new_context(E, P, w, parts_fn(), precision)
    if use_nn:
        ctx.nn_set_weights(nn[0], nn[1])
    el, prof = timed_run(ctx, w, steps, warmup, period, use_nn=use_nn,
                         kinds=("push", "push_commit"))
    pushes, iters = pushes_and_iters(prof, steps)
    r0, fb, _ = first_residuals(ctx, w, period, use_nn)
    ctx.close()
    ms = 1e3 * el / steps
    return {"precision": precision, "learned_guess": use_nn, "ms_per_step": ms,
            "s_per_step": el / steps, "particle_pushes_per_s": pushes / el,
            "picard_iterations_per_step": iters, "first_residual_mean": r0,
            "nn_fallbacks": fb, "speedup_vs_plain": plain_ms / ms}


def model_leg(E, P, w, parts_fn, steps, warmup, period, plain_ms):
    """The electrostatic model (Eq. (8)) on the same workload: the particle
    side is unchanged, the field update is the Poisson solve."""
    ctx = new_context(E, P, w, parts_fn(), "fp64", model="es")
    el, prof = timed_run(ctx, w, steps, warmup, period, kinds=("push", "push_commit", "field"))
    pushes, iters = pushes_and_iters(prof, steps)
    ctx.close()
    ms = 1e3 * el / steps
    f = prof["field"]
    return {"model": "electrostatic", "ms_per_step": ms, "particle_pushes_per_s": pushes / el,
            "picard_iterations_per_step": iters,
            "field_solve_ms": f["ms"] / f["launches"] if f["launches"] else None,
            "vs_em_step": plain_ms / ms}


# the paper's reactor feeds the drive through an annulus from 14 to 19 cm of
# radius, filled with quartz, behind a blocking capacitor (Sec. 2.1)
PORT_R_FRAC, PORT_EPS, PORT_CAP = 14.0 / 19.0, 3.8, 1e-9


def port_leg(E, P, w, parts_fn, steps, warmup, period, plain_ms):
    """The paper's drive on the same workload: the TEM port with its Mur
    condition (Eqs. (5), (7)) over the outer quarter of the bottom wall and
    the blocking capacitor (Eq. (6)); the field solve gains the port's
    coupling kernel and second scan."""
    ip = int(round(PORT_R_FRAC * (w.nr + w.xi_a) - w.xi_a))
    ctx = new_context(E, P, w, parts_fn(), "fp64", port_i=ip, port_eps=PORT_EPS,
                      blocking_cap=PORT_CAP)
    el, prof = timed_run(ctx, w, steps, warmup, period, kinds=("push", "push_commit", "field"))
    pushes, iters = pushes_and_iters(prof, steps)
    ctx.close()
    ms = 1e3 * el / steps
    f = prof["field"]
    return {"drive": "TEM port + blocking capacitor", "port_i": ip, "port_cells": w.nr - ip,
            "port_eps": PORT_EPS, "blocking_cap_F": PORT_CAP, "ms_per_step": ms,
            "particle_pushes_per_s": pushes / el, "picard_iterations_per_step": iters,
            "field_solve_ms": f["ms"] / f["launches"] if f["launches"] else None,
            "vs_gap_step": plain_ms / ms}


def jfnk_leg(E, P, w, parts_fn, steps, warmup, period, plain_ms, krylov=10, eta=1e-3):
    """The JFNK solver on the same workload, and on a dense 32x32 plasma
    (omega_pe dt = 3.4) where Picard does not converge."""
    opts = dict(solver="jfnk", krylov=krylov, eta=eta)
    ctx = new_context(E, P, w, parts_fn(), "fp64", krylov=krylov)
    el, prof = timed_run(ctx, w, steps, warmup, period, kinds=("push", "push_commit"), **opts)
    pushes, passes = pushes_and_iters(prof, steps)
    ds = [ctx.step(tol=w.tol, sort_every=period, **opts) for _ in range(4)]
    ctx.close()
    ms = 1e3 * el / steps
    out = {"solver": "jfnk", "krylov": krylov, "eta": eta, "ms_per_step": ms,
           "particle_pushes_per_s": pushes / el, "push_passes_per_step": passes,
           "newton_per_step": float(np.mean([d["newton_iters"] for d in ds])),
           "krylov_per_step": float(np.mean([d["krylov_iters"] for d in ds])),
           "vs_picard_step": plain_ms / ms}
    wd = E.workload("c1", n0=1e18, dt=6e-11, tol=1e-10)
    cd = new_context(E, P, wd, E.make_particles(wd), "fp64", krylov=20)
    d = cd.step(tol=wd.tol, max_iter=50, check=False)
    picard_rc = d["rc"]
    cd.close()
    cd = new_context(E, P, wd, E.make_particles(wd), "fp64", krylov=20)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dd = [cd.step(tol=wd.tol, max_iter=20, solver="jfnk", krylov=20, eta=1e-4)
          for _ in range(8)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cd.close()
    out["dense_32x32"] = {"omega_pe_dt": 3.38, "picard_status": picard_rc,
                          "jfnk_ms_per_step": 1e3 * el / 8,
                          "push_passes_per_step": float(np.mean([x["iters"] for x in dd])),
                          "newton_per_step": float(np.mean([x["newton_iters"] for x in dd]))}
    return out


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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_push_rate(og, E, w, n_sub, omp, passes=2):
    """Push+deposit passes of the FP64 oracle on the workload's grid over a
    sample of n_sub particles per species (uncommitted, in a random
    half-step field of a few volts plus the drive edge): particle-pushes
    per second."""
    g = og.grid_from_workload(w, omp=omp, push_only=True)
    parts = E.make_particles(w, n=n_sub, seed=w.seed + 7)
    sp = [g.species(d, cap=n_sub + 16, role=k + 1) for k, d in enumerate(parts)]
    rng = np.random.default_rng(1)
    nr, nz = w.nr, w.nz
    urh = rng.standard_normal(nr * (nz + 1)) * 3.0
    uzh = rng.standard_normal((nr + 1) * nz) * 3.0
    urh.reshape(nr, nz + 1)[:, [0, -1]] = 0
    urh.reshape(nr, nz + 1)[nr - 1, 0] = 200.0
    uzh.reshape(nr + 1, nz)[-1] = 0
    t0 = time.perf_counter()
    for _ in range(passes):
        Ir, Iz = g.zeros_r(), g.zeros_z()
        for s in sp:
            g.push_deposit(s, urh, uzh, commit=False, Ir=Ir, Iz=Iz)
    dt = time.perf_counter() - t0
    return 2 * n_sub * passes / dt, og.threads(omp)


def cpu_baseline(w):
    """The FP64 oracle on the GPU machine's host, on the same grid with a
    bounded particle sample: single-threaded, and its OpenMP build on all
    cores (particle loop in parallel, per-thread currents summed in thread
    order)."""
    import oracle as og
    import ecpic_inputs as E
    single, _ = cpu_push_rate(og, E, w, 1_000_000, omp=False)
    omp, threads = cpu_push_rate(og, E, w, 4_000_000, omp=True)
    return {"value": omp, "unit": "particle-pushes/s", "cores": threads, "kind": "oracle",
            "sample": f"2 uncommitted push+deposit passes of the FP64 oracle on the "
                      f"{w.nr}x{w.nz} grid over 4M particles per species ({threads} OpenMP "
                      f"threads; single-threaded: 1M per species), drawn by the same "
                      f"recipe from another seed, in a random half-step field",
            "single_thread": {"value": single, "cores": 1},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the mixed-precision and learned-guess legs")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned-guess legs")
    ap.add_argument("--sort-every", type=int, default=0,
                    help="steps between counting sorts (0: the workload's own cadence); "
                         "rounded down to a divisor of --steps")
    ap.add_argument("--ion-sort-stride", type=int, default=0,
                    help="the ions are sorted at every k-th of those sorts (0: the workload's "
                         "own choice)")
    ap.add_argument("--legs", default="es,port,jfnk,mixed,nn",
                    help="comma-separated legs to run beside the headline (of es, port, jfnk, "
                         "mixed, nn)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="the form of the headline leg")
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
    from paper_2212_08836_amd import nn_guess as G

    torch.cuda.set_device(0)
    w = E.workload(args.workload)
    device_gen = args.workload in ("c3", "c5")
    period = sort_period(args.steps, args.sort_every or SORT_EVERY.get(args.workload, 32))
    global SORT_STRIDES
    ion_stride = args.ion_sort_stride or ION_SORT_STRIDE.get(args.workload, 1)
    SORT_STRIDES = (1, ion_stride)
    log(f"generating the {args.workload} particles ({'GPU' if device_gen else 'host'})")
    parts = particles(E, w, device_gen)
    n0 = sum(int(len(p["r"])) for p in parts)
    ctx = new_context(E, P, w, parts, args.precision)
    del parts
    log(f"bench: {args.workload} {w.nr}x{w.nz}, {n0} particles, {args.precision}, warmup "
        f"{args.warmup}, steps {args.steps}, sort every {period}, workspace "
        f"{ctx.workspace_size() / 2**30:.1f} GiB")
    elapsed, prof = timed_run(ctx, w, args.steps, args.warmup, period)
    pushes, iters = pushes_and_iters(prof, args.steps)
    value = pushes / elapsed
    # push+deposit: the in-cell pass and the slow pass of each Picard
    # iteration (the committing iteration's pass, which also writes the
    # state and draws collisions, is reported beside it)
    fast, slow = prof["push"], prof["push_slow"]
    fast_ms = fast["ms"] / fast["launches"]
    slow_ms = slow["ms"] / slow["launches"] if slow["launches"] else 0.0
    bytes_per_pass = fast["bytes"] / fast["launches"]
    pass_ms = fast_ms + slow_ms
    achieved = bytes_per_pass / (pass_ms * 1e-3) / 1e9
    # per-kind kernel times and conservation from a short untimed run
    ctx.set_profiling(True)
    for k in range(8):
        ctx.step(tol=w.tol, sort_every=period, stats=False)
    prof_all = ctx.profile()
    ctx.set_profiling(False)
    d = ctx.step(tol=w.tol, sort_every=period, conservation=True)
    r0, _, _ = first_residuals(ctx, w, period, False)
    diag = ctx.diagnostics()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    ms = 1e3 * elapsed / args.steps
    out = {
        "metric": "particle-pushes/s per Picard iteration (and s per implicit step)",
        "value": value,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "s_per_step": elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "particles": n0,
                   "grid": [w.nr, w.nz], "dt": w.dt, "tol": w.tol,
                   "precision": args.precision, "sort_every": period,
                   "sorts_in_window": args.steps // period, "ion_sort_stride": ion_stride,
                   "parallelism": "single GPU",
                   "device_memory": "one torch tensor bound as the library's workspace"},
        "picard_iterations_per_step": iters,
        "particles_alive_end": diag["n_alive"][:2],
        "first_residual_mean": r0,
        "conservation": {"continuity_rel": d["continuity_max"] / d["q_max"],
                         "gauss_rel": d["gauss_max"] / d["q_max"]},
        "kernel_ms": {k: (v["ms"] / v["launches"] if v["launches"] else None)
                      for k, v in prof_all.items()},
        "roofline": {"bound": "hbm",
                     "kernel": "push+deposit of a Picard iteration: k_push_fast (in-cell pass) "
                               "+ k_queue (slow pass of the face crossers), both species",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": committed_traffic(args.workload, args.precision),
                     "bytes_per_pass": bytes_per_pass, "pass_ms": pass_ms,
                     "fast_ms": fast_ms, "slow_ms": slow_ms,
                     "fast_frac": bytes_per_pass / (fast_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_legs and args.precision == "fp64":
        legs = {}

        def parts_fn():
            return particles(E, w, device_gen)
        want = set(args.legs.split(","))
        if "es" in want:
            log("leg: electrostatic model")
            legs["es"] = model_leg(E, P, w, parts_fn, args.steps, args.warmup, period, ms)
            torch.cuda.empty_cache()
        if "port" in want:
            log("leg: TEM port and blocking capacitor")
            legs["port"] = port_leg(E, P, w, parts_fn, args.steps, args.warmup, period, ms)
            torch.cuda.empty_cache()
        if "jfnk" in want:
            log("leg: JFNK solver")
            legs["jfnk"] = jfnk_leg(E, P, w, parts_fn, args.steps, args.warmup, period, ms)
            torch.cuda.empty_cache()
        if "mixed" in want:
            log("leg: mixed precision, extrapolated guess")
            legs["mixed"] = leg(E, P, w, parts_fn, "mixed", False, args.steps, args.warmup,
                                period, ms)
        if not args.no_nn and "nn" in want:
            log("training the learned guess on held-out runs")
            wts, norm, info = train_network(E, P, G, w, period, device_gen)
            torch.cuda.empty_cache()
            log("leg: FP64 with the learned guess")
            legs["fp64_nn"] = leg(E, P, w, parts_fn, "fp64", True, args.steps, args.warmup,
                                  period, ms, nn=(wts, norm))
            log("leg: mixed precision with the learned guess")
            legs["mixed_nn"] = leg(E, P, w, parts_fn, "mixed", True, args.steps, args.warmup,
                                   period, ms, nn=(wts, norm))
            legs["training"] = info
        out["legs"] = legs
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
