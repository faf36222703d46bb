"""Benchmark of the GRPIC push + deposit hot path on one MI355X.

Workload (the largest single-GPU configuration): 2048 x 2048 Kerr-Schild
log-r grid (r from 0.9 r_+ to 50 r_g), spin a = 0.99, M = 1, vacuum Wald
field B0 = 1, 2e8 e+- particles (1e8 pairs placed per cell, Maxwell-Juttner
momenta at T = 0.1 m c^2 plus a 0.1c bulk rotation in phi, seed 0), dt = half
the light-crossing time of the smallest cell, ncorr = 3, particles re-sorted
by cell every 20 steps.  A step is one push + deposit of every particle (with
the sort on every 20th step), FP64.

Output: one JSON line.  value = live particle-steps per second over the timed
steps.  roofline: the push+deposit kernel's duration from HIP events on its
stream, against the binding ceiling (see the design notes); cpu_baseline: the
FP64 CPU oracle on a bounded sample of the same workload (rank 0, N = 1 only).

    python bench.py [--gpus 1] [--steps 100] [--warmup 20] [--no-cpu]
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
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, TFLOP/s

# Algorithmic HBM bytes of one FP64 particle-step: read cell (4) + xr, xth,
# ur, uth, uph, w (48) + sp (1); write cell (4) + xr, xth, ur, uth, uph (40).
FP64_PARTICLE_BYTES = 53 + 44
# Split form: cell (4) + six float32 (24) + sp (1) read; cell (4) + five float32 (20) written.
SPLIT_PARTICLE_BYTES = 29 + 24
# Algorithmic floating-point operations of one particle-step (gather, kick,
# predictor + 3 correctors, deposit), counted by running the plain CPU
# reference on a counting scalar type (+, -, *, /, sqrt, exp, sin, cos one
# each); tests/test_bench_constants.py keeps it in step with that count.
FP64_OPS_PER_PARTICLE_STEP = 1344


KERNEL_SOURCES = ("push_deposit.hip", "grpic_device.hpp", "grpic_launch.hpp")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "push_deposit_tiled_2048x2048_2e8.md")
FIELD_SOURCES = ("fields.hip", "grpic_fields.hpp", "grpic_device.hpp")
SORT_SOURCES = ("sort.hip", "grpic_launch.hpp")
SORT_TRAFFIC_PROFILE = TRAFFIC_PROFILE
FIELD_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "field_step_2048x2048.md")


def measured_traffic(profile=None, sources=None) -> dict:
    """HBM bytes per launch (or per step) from the `traffic_bytes_per_launch`
    line of a committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if the
    kernel sources are still the ones it was measured on (else empty: the
    figure is stale).  Defaults: the tiled push kernels."""
    import hashlib

    profile = profile or TRAFFIC_PROFILE
    sources = sources or KERNEL_SOURCES

    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2503_04558_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(profile) as fh:
            lines = [ln for ln in fh if ln.startswith("traffic_bytes_per_launch")]
    except OSError:
        return {}
    for line in lines:                      # the line measured on these sources, if any
        fields = dict(kv.split("=", 1) for kv in line.split()[1:])
        if fields.get("sources") == h.hexdigest():
            return {k: float(v) for k, v in fields.items() if k != "sources"}
    return {}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(npairs: int, nr: int, nth: int, a: float, device: str = "cuda", workers: int = 16):
    import torch

    from paper_2503_04558_amd import grpic
    from paper_2503_04558_amd import workload as wl

    g = wl.make_grid(nr, nth, a)
    F = [torch.as_tensor(f).to(device) for f in wl.wald_fields(g, B0=1.0)]
    n = 2 * npairs
    parts = grpic.empty_particles(n, device=device)

    def sink(start, arrs):
        m = len(arrs["cell"])
        for k, v in arrs.items():
            parts[k][start:start + m].copy_(torch.from_numpy(np.ascontiguousarray(v)))

    wl.pairs(g, npairs, kind="mj", seed=0, params=dict(T=0.1, vphi=0.1), workers=workers, sink=sink)
    return g, F, parts


def run_gpu(args, g, F, parts, precision, kick="boris"):
    """Warm up, then time args.steps push + deposit steps of one precision
    (and kick: the generalised Boris kick, or Vay's in the FIDO frame)."""
    import torch

    from paper_2503_04558_amd import grpic
    from paper_2503_04558_amd import workload as wl

    dev = "cuda"
    sp = wl.species_table()
    metric = grpic.make_metric(g.a, g.M)
    dt = 0.5 * grpic.grpic_crossing_time(metric, g)
    J = [torch.zeros(g.shape, dtype=torch.float64, device=dev) for _ in range(3)]
    counters = torch.zeros(grpic.GRPIC_NCOUNTERS, dtype=torch.int64, device=dev)
    sorter = grpic.Sorter(g, parts["cell"].numel(), precision, device=dev)
    state = {"p": parts}

    def do_sort():
        state["p"] = sorter.sort(state["p"])

    ev_push = []
    ev_sort = []

    def step(k, timed):
        if k % args.sort_every == 0:
            if timed:
                s0 = torch.cuda.Event(enable_timing=True)
                s1 = torch.cuda.Event(enable_timing=True)
                s0.record()
            do_sort()
            if timed:
                s1.record()
                ev_sort.append((s0, s1))
        if timed:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        grpic.grpic_push_deposit(metric, g, sp, state["p"], F, J, dt, 1, args.ncorr, tiling=sorter.tiling,
                                 counters=counters if timed else None, kick=kick)
        if timed:
            e1.record()
            ev_push.append((e0, e1))

    for k in range(args.warmup):
        step(k, False)
    torch.cuda.synchronize()
    label = ('split' if precision else 'fp64') + ('' if kick == 'boris' else f' ({kick} kick)')
    log(f"{label}: warmup {args.warmup} steps done")
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.time()
    start.record()
    for k in range(args.warmup, args.warmup + args.steps):
        step(k, True)
    stop.record()
    torch.cuda.synchronize()
    t_wall = time.time() - t_wall
    total_ms = start.elapsed_time(stop)
    push_ms = [a.elapsed_time(b) for a, b in ev_push]
    sort_ms = [a.elapsed_time(b) for a, b in ev_sort]
    cnt = dict(zip(grpic.COUNTER_NAMES, counters.cpu().tolist()))
    log(f"{label}: timed {args.steps} steps: {total_ms:.2f} ms (wall {t_wall:.2f}s), "
        f"counters {cnt}")
    live = cnt["live_steps"]
    value = live / (total_ms * 1e-3)
    avg_push_ms = float(np.mean(push_ms))
    # roofline of the push + deposit kernel (one launch per step)
    live_per_launch = live / args.steps
    field_bytes = 8 if precision == grpic.GRPIC_FP64 else 4
    grid_bytes = g.rows * g.pitch * (6 * field_bytes + 2 * 3 * 8)   # fields read once, J read + written once
    pbytes = FP64_PARTICLE_BYTES if precision == grpic.GRPIC_FP64 else SPLIT_PARTICLE_BYTES
    bytes_per_launch = live_per_launch * pbytes + grid_bytes
    hbm_gbs = bytes_per_launch / (avg_push_ms * 1e-3) / 1e9
    flops_per_launch = live_per_launch * FP64_OPS_PER_PARTICLE_STEP
    tflops = flops_per_launch / (avg_push_ms * 1e-3) / 1e12
    return dict(value=value, total_ms=total_ms, avg_push_ms=avg_push_ms, push_ms=push_ms, sort_ms=sort_ms, counters=cnt,
                hbm_gbs=hbm_gbs, bytes_per_launch=bytes_per_launch, dt=dt, live_per_launch=live_per_launch,
                wall_s=t_wall, tflops=tflops, flops_per_launch=flops_per_launch)


def run_adjoint(args):
    """Backward / forward time of K = 32 FP64 steps (checkpoints every 8) on a
    512 x 512 grid (a = 0.9, Wald B0 = 1) with 1e6 Maxwell-Juttner particles
    (T = 0.5); loss: the charge carried through the shell r = 5.  Forward: the
    sorted, tiled push of the K steps in one call, with and without saving the
    checkpoints; backward: grpic_push_deposit_backward."""
    import torch

    from paper_2503_04558_amd import grpic
    from paper_2503_04558_amd import workload as wl

    K, C = 32, 8
    g = wl.make_grid(512, 512, 0.9)
    F = [torch.as_tensor(f).to("cuda") for f in wl.wald_fields(g, B0=1.0)]
    parts = grpic.to_device(wl.pairs(g, args.adj_pairs, kind="mj", seed=0, params=dict(T=0.5),
                                     workers=args.workers))
    sp = wl.species_table()
    metric = grpic.make_metric(g.a, g.M)
    dt = wl.crossing_dt(g)
    n = parts["cell"].numel()
    sorter = grpic.Sorter(g, n, grpic.GRPIC_FP64)
    start = sorter.sort(parts)
    start = {k: v.clone() for k, v in start.items()}
    i = np.arange(g.nr)
    face = int(np.argmin(np.abs(g.r(i + 0.5) - 5.0)))
    lam = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    lam[0][g.guard + face, :] = dt
    ck = torch.empty(grpic.grpic_checkpoint_bytes(n, K, C), dtype=torch.uint8, device="cuda")
    ws = torch.empty(grpic.grpic_backward_workspace_bytes(g, n, C), dtype=torch.uint8, device="cuda")
    gu = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    gF = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(6)]
    J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def fwd(with_ckpt):
        p = {k: v.clone() for k, v in start.items()}
        torch.cuda.synchronize()
        return timed(lambda: grpic.grpic_push_deposit(metric, g, sp, p, F, J, dt, K, args.ncorr,
                                                      tiling=sorter.tiling, ckpt=ck if with_ckpt else None,
                                                      ckpt_every=C if with_ckpt else 0))

    # a dense cotangent (every grid entry non-zero) for comparison: no step can be skipped
    gen = torch.Generator(device="cuda").manual_seed(0)
    lam_dense = [torch.randn(g.shape, dtype=torch.float64, device="cuda", generator=gen) * dt for _ in range(3)]

    def bwd(lm):
        return timed(lambda: grpic.grpic_push_deposit_backward(metric, g, sp, start, F, lm, dt, K, args.ncorr, ck,
                                                               C, ws, gu, gF))

    fwd(True), bwd(lam)                    # warm-up
    f_plain = [fwd(False) for _ in range(3)]
    f_ck = [fwd(True) for _ in range(3)]
    b = [bwd(lam) for _ in range(3)]
    bd = [bwd(lam_dense) for _ in range(2)]
    log(f"adjoint: fwd {f_plain} ms, fwd+ckpt {f_ck} ms, bwd {b} ms, bwd dense lambda {bd} ms")
    return {"workload": f"512x512, a=0.9, Wald B0=1, {n} particles (Maxwell-Juttner T=0.5), K={K} steps, "
                        f"checkpoints every {C}, loss = charge through r=5",
            "fwd_ms": min(f_plain), "fwd_ckpt_ms": min(f_ck), "bwd_ms": min(b),
            "bwd_over_fwd": min(b) / min(f_ck),
            "dense_lambda_bwd_ms": min(bd), "dense_lambda_bwd_over_fwd": min(bd) / min(f_ck)}


# Field step: grid planes one evaluation must move at least, with the
# metric coefficients formed in registers, the six inverse areas tabulated
# and the corrector's constant part R = X^n + dt (w0 C(X^n) - J) formed once:
# the predictor reads the state, inverse areas and currents (3) and writes
# the predicted state and R; a corrector pass reads the iterate, R and the
# inverse areas and writes the iterate.
FIELD_PLANES_PREDICTOR = 6 + 6 + 3 + 6 + 6
FIELD_PLANES_CORRECTOR = 6 + 6 + 6 + 6


def run_fields(args, g, F):
    """Time field steps (predictor + args.field_ncorr correctors) of the
    Wald state on the throughput grid, currents passed (zero), damping over
    the outer 64 rows."""
    import torch

    from paper_2503_04558_amd import grpic

    metric = grpic.make_metric(g.a, g.M)
    dt = 0.5 * grpic.grpic_crossing_time(metric, g)
    solver = grpic.FieldSolver(metric, g)
    state = [f.to(torch.float64).clone() for f in F]
    J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    stream = torch.cuda.current_stream()
    kw = dict(w1=args.field_w1, ncorr=args.field_ncorr, damp_cells=64, damp_max=0.05)
    for _ in range(2):
        solver.step(state, J, dt, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.field_steps):
        solver.step(state, J, dt, stream=stream, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.field_steps
    finite = all(bool(torch.isfinite(s).all()) for s in state)
    plane = (g.nr + 1) * (g.nth + 1) * 8
    nbytes = plane * (FIELD_PLANES_PREDICTOR + args.field_ncorr * FIELD_PLANES_CORRECTOR)
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"fields: {args.field_steps} steps of ncorr={args.field_ncorr}: {ms:.3f} ms/step, finite={finite}")
    return {"grid": [g.nr, g.nth], "ncorr": args.field_ncorr, "w1": args.field_w1, "steps": args.field_steps,
            "ms_per_step": ms, "cell_updates_per_s": g.nr * g.nth / (ms * 1e-3), "finite": finite,
            "roofline_hbm": dict(bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                                 frac=round(gbs / HBM_PEAK_GBS, 4),
                                 traffic=measured_traffic(FIELD_TRAFFIC_PROFILE, FIELD_SOURCES).get("step"),
                                 bytes_per_step=nbytes)}


# A re-sort reads each particle's cell for the histogram (4 B), then its
# cell and state (FP64: 5 x 8 B + weight 8 B + species 1 B + cell 4 B =
# 53 B) and writes them at their sorted position (53 B).
SORT_BYTES_PER_PARTICLE_F64 = 4 + 53 + 53


def _sort_roofline(sort_ms, n, per_particle, traffic=None):
    """HBM roofline of the timed re-sorts (the drifted order of a running
    simulation; the first sort of the generator's random order is untimed).
    traffic: the measured HBM bytes of one re-sort (all its kernels), if the
    sources still match the profile."""
    if not sort_ms:
        return None
    ms = float(np.mean(sort_ms))
    gbs = n * per_particle / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                traffic=traffic, bytes_per_sort=n * per_particle, avg_ms=ms)


def run_pic(args, steps: int, warmup: int) -> dict:
    """The full-step batch in the FP32-split form: on a pic_grid^2 grid
    (a = 0.99), 2 * pic_pairs e+- with dN/dgamma ~ gamma^-2 on [1, 1e3]
    (seed 0) and the Wald field B0 = 1 as the initial state, each step is a
    tiled split push + deposit against a float copy of the fields, then the
    field step (predictor + 7 correctors, w1 = 0.53, damping over the outer
    32 rows) with that step's currents; re-sorted every sort_every steps.
    Returns the time per PIC step and its parts (HIP events)."""
    import torch

    from paper_2503_04558_amd import grpic
    from paper_2503_04558_amd import workload as wl

    t0 = time.time()
    g = wl.make_grid(args.pic_grid, args.pic_grid, 0.99)
    n = 2 * args.pic_pairs
    parts = grpic.empty_particles(n, grpic.GRPIC_FP32_SPLIT)

    def sink(start, arrs):
        m = len(arrs["cell"])
        for k, v in arrs.items():
            parts[k][start:start + m].copy_(torch.from_numpy(np.ascontiguousarray(v)))

    wl.pairs(g, args.pic_pairs, kind="powerlaw", seed=0, params=dict(gmax=1e3), workers=args.workers, sink=sink)
    state = [torch.as_tensor(f).cuda() for f in wl.wald_fields(g, B0=1.0)]
    torch.cuda.synchronize()
    log(f"pic: inputs ready in {time.time() - t0:.1f}s: grid {g.nr}x{g.nth}, {n} split particles")
    sp = wl.species_table()
    metric = grpic.make_metric(g.a, g.M)
    dt = 0.5 * grpic.grpic_crossing_time(metric, g)
    sorter = grpic.Sorter(g, n, grpic.GRPIC_FP32_SPLIT)
    solver = grpic.FieldSolver(metric, g)
    F32 = [s.float() for s in state]
    J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    counters = torch.zeros(grpic.GRPIC_NCOUNTERS, dtype=torch.int64, device="cuda")
    cur = {"p": parts}
    marks = []

    def step(k, timed):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if timed else None
        if timed:
            ev[0].record()
        if k % args.sort_every == 0:
            cur["p"] = sorter.sort(cur["p"])
        if timed:
            ev[1].record()
        for j in J:
            j.zero_()
        for f32, s in zip(F32, state):
            f32.copy_(s)
        if timed:
            ev[2].record()
        grpic.grpic_push_deposit(metric, g, sp, cur["p"], F32, J, dt, 1, args.ncorr, tiling=sorter.tiling,
                                 counters=counters if timed else None)
        if timed:
            ev[3].record()
        solver.step(state, J, dt, 0.53, 7, damp_cells=32, damp_max=0.1)
        if timed:
            ev[4].record()
            marks.append(ev)

    for k in range(warmup):
        step(k, False)
    torch.cuda.synchronize()
    w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0.record()
    for k in range(warmup, warmup + steps):
        step(k, True)
    w1.record()
    torch.cuda.synchronize()
    total = w0.elapsed_time(w1)
    part = np.array([[m[i].elapsed_time(m[i + 1]) for i in range(4)] for m in marks])
    cnt = dict(zip(grpic.COUNTER_NAMES, counters.cpu().tolist()))
    finite = all(bool(torch.isfinite(s).all()) for s in state)
    live = cnt["live_steps"] / steps
    out = {"metric": "full PIC step (split push + deposit + field step) particle-steps/s", "unit": "particle-steps/s",
           "value": cnt["live_steps"] / (total * 1e-3), "ms_per_step": total / steps, "steps": steps,
           "warmup": warmup, "dtype": "f32 particles and fields for the push (f64 in r < 2M, near the axis, "
           "and for the deposit); f64 field solver",
           "config": {"workload": f"{g.nr}x{g.nth} Kerr-Schild log-r grid, a=0.99, {n} e+- (dN/dgamma ~ gamma^-2 "
                                  f"on [1, 1e3]), Wald B0=1 initial fields, field step N=7 w1=0.53, sort every "
                                  f"{args.sort_every} steps, ncorr={args.ncorr}", "dt": dt},
           "parts_ms": {"sort_avg_per_step": float(part[:, 0].mean()), "zero_J_and_float_fields": float(part[:, 1].mean()),
                        "push_deposit": float(part[:, 2].mean()), "field_step": float(part[:, 3].mean())},
           "live_particles_per_step": live, "counters": cnt, "fields_finite": finite}
    log(f"pic: {out['ms_per_step']:.2f} ms per PIC step, parts {out['parts_ms']}")
    if args.pic_adj_steps > 0:
        out["adjoint"] = pic_adjoint(args, g, metric, sp, dt, cur, sorter, solver, state, F32, J)
    del parts, cur, sorter, solver, state, F32, J
    torch.cuda.empty_cache()
    return out


def pic_adjoint(args, g, metric, sp, dt, cur, sorter, solver, state, F32, J) -> dict:
    """The adjoint over the next pic_adj_steps PIC steps of the full-step
    batch: after a re-sort, each step saves the field state its push gathers
    from (FP64) and, every pic_adj_every steps, a checkpoint of the split
    particles promoted to FP64; then grpic_push_deposit_backward_range
    reverses the window in batches of pic_adj_batch particles (one bounded
    workspace) with those per-step fields, for the charge carried through
    the shell r = 5.  Times: the window's pushes (with the checkpoint saves),
    its full PIC steps, and the backward."""
    import torch

    from paper_2503_04558_amd import grpic

    K, C = args.pic_adj_steps, args.pic_adj_every
    cur["p"] = sorter.sort(cur["p"])
    p = cur["p"]
    n = p["cell"].numel()
    slot = grpic.grpic_checkpoint_bytes(n, 1, 1)
    ck = torch.empty(K // C * slot, dtype=torch.uint8, device="cuda")
    hist = torch.empty((6, K) + tuple(g.shape), dtype=torch.float64, device="cuda")
    Jsum = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0.record()
    for k in range(K):
        for c in range(6):
            hist[c, k].copy_(state[c])
        for j in J:
            j.zero_()
        for f32, s_ in zip(F32, state):
            f32.copy_(s_)
        kw = dict(ckpt=ck[(k // C) * slot:(k // C + 1) * slot], ckpt_every=1) if k % C == 0 else {}
        ev[k][0].record()
        grpic.grpic_push_deposit(metric, g, sp, p, F32, J, dt, 1, args.ncorr, tiling=sorter.tiling, **kw)
        ev[k][1].record()
        for a, b in zip(Jsum, J):
            a += b
        solver.step(state, J, dt, 0.53, 7, damp_cells=32, damp_max=0.1)
    w1.record()
    torch.cuda.synchronize()
    fwd_push_ms = sum(a.elapsed_time(b) for a, b in ev)
    fwd_pic_ms = w0.elapsed_time(w1)
    i_star = int(np.argmin(np.abs(g.r(np.arange(g.nr) + 0.5) - 5.0)))
    lam = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    lam[0][g.guard + i_star, :] = dt
    L = sum(float((l * j).sum()) for l, j in zip(lam, Jsum))
    del Jsum
    # the backward reads w and sp (as FP64); the sort spare is not needed now
    view = {"w": p["w"].double(), "sp": p["sp"]}
    batch = min(n, args.pic_adj_batch)
    ws = torch.empty(grpic.grpic_backward_workspace_bytes(g, batch, C), dtype=torch.uint8, device="cuda")
    gu = [torch.empty(batch, dtype=torch.float64, device="cuda") for _ in range(3)]
    plane = g.rows * g.pitch
    nonzero = 0
    gmax = 0.0
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b0.record()
    for first in range(0, n, batch):
        cnt = min(batch, n - first)
        grpic.grpic_push_deposit_backward_range(metric, g, sp, view, [hist[c, 0] for c in range(6)], lam, dt, K,
                                                args.ncorr, ck, C, first, cnt, ws, [t[:cnt] for t in gu],
                                                field_step_stride=plane)
        a = torch.stack([t[:cnt] for t in gu]).abs().amax(dim=0)
        nonzero += int((a > 0).sum())
        gmax = max(gmax, float(a.max()))
    b1.record()
    torch.cuda.synchronize()
    bwd_ms = b0.elapsed_time(b1)
    finite = all(bool(torch.isfinite(t).all()) for t in gu)
    res = {"steps": K, "ckpt_every": C, "batch": batch, "batches": (n + batch - 1) // batch,
           "fwd_push_ms": fwd_push_ms, "fwd_pic_ms": fwd_pic_ms, "bwd_ms": bwd_ms,
           "bwd_over_fwd_push": bwd_ms / fwd_push_ms, "bwd_over_fwd_pic": bwd_ms / fwd_pic_ms,
           "loss": "charge through the shell r = 5 over the window", "L": L, "particles": n,
           "nonzero_gradients": nonzero, "max_abs_gradient": gmax, "finite": finite,
           "memory": {"checkpoints_gb": ck.numel() / 1e9, "field_history_gb": hist.numel() * 8 / 1e9,
                      "workspace_gb": ws.numel() / 1e9}}
    log(f"pic adjoint: {res}")
    del ck, hist, view, ws, gu, lam
    torch.cuda.empty_cache()
    return res


def run_qed(args) -> dict:
    """The monopole workload (Sec. 4): on the throughput grid, the vacuum
    monopole of App. C with B0 = 2e3 (D from the 3+1 relations), 2 * qed_pairs
    particles of the full-step batch's power-law recipe with a fifth of the
    pairs' e- slots turned into photons (FIDO energy uniform in [1, 10]);
    gamma_thr = 100, eps_ph = 4, tau = 2, dt = 5e-4; arrays with room for
    twice the initial count; grpic_push_deposit_qed with its staging
    workspace, re-sorted every sort_every steps (the sort's live count feeds
    the step's count of elements in use)."""
    import torch

    from paper_2503_04558_amd import grpic
    from paper_2503_04558_amd import workload as wl

    t0 = time.time()
    g = wl.make_grid(args.nr, args.nth, args.spin)
    n0 = 2 * args.qed_pairs
    cap = 2 * n0
    parts = grpic.empty_particles(cap, with_tag=True)
    parts["cell"].fill_(-1)
    host = wl.qed_particles(g, args.qed_pairs, seed=0, workers=args.workers)
    host["tag"] = host["tag"].view(np.int64)
    for k, v in host.items():
        parts[k][:n0].copy_(torch.from_numpy(np.ascontiguousarray(v)))
    del host
    F = [torch.as_tensor(f).cuda() for f in wl.monopole_fields(g, B0=2e3)]
    torch.cuda.synchronize()
    log(f"qed: inputs ready in {time.time() - t0:.1f}s: {n0} particles, capacity {cap}")
    sp = wl.qed_species_table()
    metric = grpic.make_metric(g.a, g.M)
    dt = 5e-4
    qed = grpic.make_qed(100.0, 4.0, 2.0, seed=0)
    sorter = grpic.Sorter(g, cap, with_tag=True)
    ws = torch.empty(grpic.grpic_qed_workspace_bytes(g, cap), dtype=torch.uint8, device="cuda")
    n_used = torch.tensor([n0, 0], dtype=torch.int64, device="cuda")
    J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    counters = torch.zeros(grpic.GRPIC_NCOUNTERS, dtype=torch.int64, device="cuda")
    qc = torch.zeros(grpic.GRPIC_NQCOUNTERS, dtype=torch.int64, device="cuda")
    cur = {"p": parts}

    def step(k, timed):
        if k % args.sort_every == 0:
            cur["p"] = sorter.sort(cur["p"])
            n_used[:1].copy_(sorter.n_alive)
        grpic.grpic_push_deposit_qed(metric, g, sp, cur["p"], F, J, dt, k, qed, n_used, args.ncorr,
                                     tiling=sorter.tiling, ws=ws, counters=counters if timed else None,
                                     qcounters=qc if timed else None)

    for k in range(args.qed_warmup):
        step(k, False)
    torch.cuda.synchronize()
    start_n = int(n_used[0].item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.qed_warmup, args.qed_warmup + args.qed_steps):
        step(k, True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cnt = dict(zip(grpic.COUNTER_NAMES, counters.cpu().tolist()))
    q = dict(zip(grpic.QCOUNTER_NAMES, qc.cpu().tolist()))
    out = {"value": cnt["live_steps"] / (ms * 1e-3), "unit": "particle-steps/s", "dtype": "f64",
           "ms_per_step": ms / args.qed_steps, "steps": args.qed_steps, "warmup": args.qed_warmup,
           "config": {"workload": f"{g.nr}x{g.nth} Kerr-Schild log-r grid, a={g.a}, vacuum monopole B0=2e3, "
                                  f"{n0} e+- and photons (dN/dgamma ~ gamma^-2 on [1, 1e3], 20% of the pairs' e- "
                                  f"slots photons), gamma_thr=100, eps_ph=4, tau=2, dt=5e-4, sort every "
                                  f"{args.sort_every} steps", "capacity": cap},
           "elements_in_use": [start_n, int(n_used[0].item())], "events": q, "counters": cnt}
    log(f"qed: {out['ms_per_step']:.2f} ms/step, events {q}, in use {out['elements_in_use']}")
    del parts, cur, sorter, F, J, ws
    torch.cuda.empty_cache()
    return out


def run_spline3(args) -> dict:
    """The third-order (cubic spline) shape against CIC on the same
    particles and fields: 2 * spline_pairs e+- of the throughput recipe on
    the 2048^2 grid with guard 3, untiled (generator order) and tiled (after
    a GPU sort); 1 warm-up and args.spline_steps timed steps each, HIP
    events on the launch stream."""
    import torch

    from paper_2503_04558_amd import grpic
    from paper_2503_04558_amd import workload as wl

    g = wl.make_grid(args.nr, args.nth, args.spin, guard=3)
    host = wl.pairs(g, args.spline_pairs, kind="mj", seed=0, params=dict(T=0.1, vphi=0.1), workers=args.workers)
    F = [torch.as_tensor(f).cuda() for f in wl.wald_fields(g, B0=1.0)]
    sp = wl.species_table()
    metric = grpic.make_metric(g.a, g.M)
    dt = 0.5 * grpic.grpic_crossing_time(metric, g)
    n = 2 * args.spline_pairs
    out = {}
    for tiled in (False, True):
        for order in (3, 1):
            parts = grpic.to_device(host)
            tiling = None
            if tiled:
                sorter = grpic.Sorter(g, n, grpic.GRPIC_FP64)
                parts = sorter.sort(parts)
                tiling = sorter.tiling
            J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
            counters = torch.zeros(grpic.GRPIC_NCOUNTERS, dtype=torch.int64, device="cuda")
            grpic.grpic_push_deposit(metric, g, sp, parts, F, J, dt, 1, args.ncorr, tiling=tiling, order=order)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            grpic.grpic_push_deposit(metric, g, sp, parts, F, J, dt, args.spline_steps, args.ncorr, tiling=tiling,
                                     counters=counters, order=order)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.spline_steps
            live = counters.cpu().tolist()[grpic.COUNTER_NAMES.index("live_steps")] / args.spline_steps
            out[(tiled, order)] = dict(ms_per_step=ms, value=live / (ms * 1e-3))
            del parts, J
    log(f"spline3: tiled {out[(True, 3)]['ms_per_step']:.2f} ms/step (CIC tiled {out[(True, 1)]['ms_per_step']:.2f}), "
        f"untiled {out[(False, 3)]['ms_per_step']:.2f} (CIC untiled {out[(False, 1)]['ms_per_step']:.2f})")
    t3, t1 = out[(True, 3)], out[(True, 1)]
    return {"value": t3["value"], "unit": "particle-steps/s", "dtype": "f64", "ms_per_step": t3["ms_per_step"],
            "kernel": "push_deposit_f64_tiled_spline3", "particles": n, "vs_cic_tiled": t3["value"] / t1["value"],
            "cic_tiled_same_particles": t1, "untiled": out[(False, 3)], "cic_untiled_same_particles": out[(False, 1)]}


def copy_ceiling_gbs(gib: int = 4, reps: int = 5) -> dict:
    """A STREAM ceiling measured on this GPU over a gib-GiB FP64 array (read +
    write counted): the runtime's device-to-device copy, and STREAM's scale
    (b = 1.0 * a, torch's vectorised elementwise kernel); HIP events around
    reps passes after two warm-ups.  The ceiling is the faster of the two."""
    import torch

    a = torch.ones(gib * (1 << 30) // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    nbytes = 2 * a.numel() * 8
    out = {}
    for name, op in (("copy", lambda: b.copy_(a)), ("scale", lambda: torch.mul(a, 1.0, out=b))):
        for _ in range(2):
            op()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            op()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    best = max(out.values())
    return {"achieved": best, "unit": "GB/s", "frac_of_peak": round(best / HBM_PEAK_GBS, 4),
            "bytes_per_pass": nbytes, **{f"{k}_gbs": v for k, v in out.items()}}


def usable_cpus() -> int:
    """CPUs this process may run on (its affinity set: the host's share)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def split_error_report(args, grid, parts, F, dt, orc) -> dict:
    """The split form's stated error on a sample of the workload's own
    particles: the first args.split_sample of them, rounded to float, 10
    steps of the FP32-split push on the GPU (float fields) against the FP64
    oracle from the same float-representable state (FP64 fields).  Momentum:
    max_i |d u_i| sqrt(gamma^ii) / sqrt(1 + u^2) per particle; energy:
    |dE_split - dE_oracle| / max(1, |terms|) with E = alpha sqrt(1 + u^2) -
    beta^r u_r - (q/m) A_t; continuity: max per vertex of |Q^10 - Q^0 + dt
    div F| over sum |q w| on the GPU's own outputs, in units of eps.  As in
    the parity tests, the maxima are over the particles whose response to
    one float rounding of their state (the oracle run again on it) stays
    below an eighth of the bar; the others are counted, and every particle
    must lie within the bar plus 64 times its own response."""
    import torch

    from paper_2503_04558_amd import grpic
    from paper_2503_04558_amd import workload as wl

    nsteps = 10
    m = args.split_sample
    p0 = {k: np.asarray(v[:m], dtype=np.float32).astype(np.float64) if k in grpic.REAL_KEYS else v[:m].copy()
          for k, v in parts.items()}
    sp = wl.species_table()
    po, _, _, _ = orc.run(grid, sp, p0, F, dt, nsteps, ncorr=args.ncorr, nthreads=usable_cpus())
    # each particle's rounding sensitivity: the oracle's response to moving
    # its float state by one float rounding (2^-24)
    rng = np.random.default_rng(7)
    pq = {k: np.array(v, copy=True) for k, v in p0.items()}
    for k in ("xr", "xth"):
        pq[k] = np.clip(pq[k] + rng.choice([-1.0, 1.0], m) * 2.0 ** -24, 0.0, 1.0 - 2.0 ** -52)
    for k in ("ur", "uth", "uph"):
        pq[k] = pq[k] * (1.0 + rng.choice([-1.0, 1.0], m) * 2.0 ** -24)
    pp, _, _, _ = orc.run(grid, sp, pq, F, dt, nsteps, ncorr=args.ncorr, nthreads=usable_cpus())
    dev = grpic.to_device(p0, grpic.GRPIC_FP32_SPLIT)
    F32 = [torch.as_tensor(f).to(device="cuda", dtype=torch.float32) for f in F]
    J = [torch.zeros(grid.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    Q0 = torch.zeros(grid.shape, dtype=torch.float64, device="cuda")
    Q1 = torch.zeros_like(Q0)
    grpic.grpic_charge(grid, sp, dev, Q0)
    grpic.grpic_push_deposit(grpic.make_metric(grid.a, grid.M), grid, sp, dev, F32, J, dt, nsteps, args.ncorr)
    grpic.grpic_charge(grid, sp, dev, Q1)
    div = torch.zeros_like(J[0])
    div[1:, :] += J[0][1:, :] - J[0][:-1, :]
    div[:, 1:] += J[1][:, 1:] - J[1][:, :-1]
    R = (Q1 - Q0 + dt * div)[grid.guard + 1: grid.guard + grid.nr]
    cont = R.abs().max().item() / (dev["w"].abs().sum().item() * np.finfo(np.float64).eps)
    pg = {k: np.asarray(v, dtype=np.float64) if k not in ("cell", "sp") else v for k, v in grpic.to_host(dev).items()}
    live = (pg["cell"] >= 0) & (po["cell"] >= 0)

    def state(p):
        ci, cj = p["cell"] // grid.nth, p["cell"] % grid.nth
        xi, eta = ci + p["xr"], cj + p["xth"]
        k = wl._ks_pieces(grid.a, grid.M, grid.r(xi), grid.theta(eta))
        u = [p[c] for c in ("ur", "uth", "uph")]
        with np.errstate(invalid="ignore", over="ignore"):
            uu = k["h_rr"] * u[0] ** 2 + 2 * k["h_rp"] * u[0] * u[2] + k["h_tt"] * u[1] ** 2 + k["h_pp"] * u[2] ** 2
            qm = np.where(p["sp"] == 0, -1.0, 1.0)
            At = wl.wald_point(grid.a, grid.M, 1.0, grid.r(xi), grid.theta(eta))["At"]
            terms = (k["alpha"] * np.sqrt(1 + uu), -k["beta"] * u[0], -qm * At)
        return k, u, uu, terms[0] + terms[1] + terms[2], np.abs(terms[0]) + np.abs(terms[1]) + np.abs(terms[2])

    ko, uo, uuo, Eo, so = state(po)
    _, ug, _, Eg, sg = state(pg)
    _, up, _, Ep, _ = state(pp)
    _, _, _, E0, s0 = state(p0)
    _, _, _, Eq0, _ = state(pq)
    with np.errstate(invalid="ignore", divide="ignore"):
        def mom_err(u):
            return np.max([np.abs(u[i] - uo[i]) * np.sqrt(ko[h]) for i, h in enumerate(("h_rr", "h_tt", "h_pp"))],
                          axis=0) / np.sqrt(1.0 + uuo)
        scale = np.maximum(np.maximum(np.maximum(s0, so), sg), 1.0)
        mom, mom_s = mom_err(ug), mom_err(up)
        en = np.abs((Eg - E0) - (Eo - E0)) / scale
        en_s = np.abs((Ep - Eq0) - (Eo - E0)) / scale
    live &= (pp["cell"] >= 0)
    tol = 1e-5
    ill = (mom_s > tol / 8) | (en_s > tol / 8)          # rounding-sensitive beyond an eighth of the bar
    good = live & ~ill
    return {"sample": f"first {m} particles of the workload, float-representable, {nsteps} steps, untiled",
            "momentum_max": float(mom[good].max()), "momentum_median": float(np.median(mom[good])),
            "energy_max": float(en[good].max()), "energy_median": float(np.median(en[good])),
            "ill_conditioned": int((live & ill).sum()),
            "momentum_max_all": float(mom[live].max()), "energy_max_all": float(en[live].max()),
            "violations": int(np.count_nonzero((mom[live] > tol + 64 * mom_s[live])
                                               | (en[live] > tol + 64 * en_s[live]))),
            "continuity_max_eps": float(cont), "live": int(live.sum()),
            "status_mismatch": int(np.count_nonzero((pg["cell"] >= 0) != (po["cell"] >= 0)
                                                    & ((pp["cell"] >= 0) == (po["cell"] >= 0)))),
            "stated": {"momentum": tol, "energy": tol, "continuity_eps": 64,
                       "conditioning": "maxima over particles whose one-rounding sensitivity is below 1/8 of "
                                       "the bar; every particle must be within the bar plus 64 times it"}}


def run_cpu_baseline(args, grid):
    """The FP64 oracle (OpenMP over particles) on a bounded sample, on every
    CPU this process may use; its run on the sample's first particles is also
    the reference of the split form's error report."""
    from oracle import oracle as orc
    from paper_2503_04558_amd import workload as wl

    nthreads = usable_cpus()
    sample_pairs = args.cpu_pairs
    parts = wl.pairs(grid, sample_pairs, kind="mj", seed=0, params=dict(T=0.1, vphi=0.1), workers=nthreads)
    F = wl.wald_fields(grid, B0=1.0)
    dt = wl.crossing_dt(grid)
    split = None
    if not args.no_split:
        try:
            split = split_error_report(args, grid, parts, F, dt, orc)
        except Exception as e:                        # noqa: BLE001 -- reported in the JSON line
            split = {"error": repr(e)}
        log(f"split error report: {split}")
    t = time.time()
    _, _, _, st = orc.run(grid, wl.species_table(), parts, F, dt, args.cpu_steps, ncorr=args.ncorr,
                          nthreads=nthreads)
    el = time.time() - t
    rate = st["live_steps"] / el
    # one thread, on the first 1/64 of the sample
    small = {k: v[: len(v) // 64] for k, v in parts.items()}
    t = time.time()
    _, _, _, st1 = orc.run(grid, wl.species_table(), small, F, dt, args.cpu_steps, ncorr=args.ncorr, nthreads=1)
    el1 = time.time() - t
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=rate, unit="particle-steps/s", cores=nthreads if orc.has_openmp() else 1, kind="oracle",
                sample=f"first {2 * sample_pairs} particles of the same workload, {args.cpu_steps} steps, "
                       f"no sort, {el:.1f}s",
                one_thread_value=st1["live_steps"] / el1, host_cpus=os.cpu_count(), cpu_model=model,
                split_error=split)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--pairs", type=int, default=100_000_000)
    ap.add_argument("--nr", type=int, default=2048)
    ap.add_argument("--nth", type=int, default=2048)
    ap.add_argument("--spin", type=float, default=0.99)
    ap.add_argument("--ncorr", type=int, default=3)
    ap.add_argument("--sort-every", type=int, default=20)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-split", action="store_true", help="skip the FP32-split timing")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the backward / forward timing")
    ap.add_argument("--adj-pairs", type=int, default=500_000)
    ap.add_argument("--no-fields", action="store_true", help="skip the field-solver timing")
    ap.add_argument("--no-vay", action="store_true", help="skip the timing of the push with Vay's kick")
    ap.add_argument("--no-spline3", action="store_true", help="skip the timing of the cubic spline shape")
    ap.add_argument("--spline-pairs", type=int, default=10_000_000)
    ap.add_argument("--spline-steps", type=int, default=5)
    ap.add_argument("--field-steps", type=int, default=10)
    ap.add_argument("--field-ncorr", type=int, default=7)
    ap.add_argument("--field-w1", type=float, default=0.53)
    ap.add_argument("--cpu-pairs", type=int, default=5_000_000)
    ap.add_argument("--split-sample", type=int, default=1_000_000)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--pic", action="store_true",
                    help="only time the full PIC step of the split-form batch (push + deposit + field step)")
    ap.add_argument("--no-pic", action="store_true", help="skip the full PIC step leg")
    ap.add_argument("--pic-grid", type=int, default=4096)
    ap.add_argument("--pic-pairs", type=int, default=500_000_000)
    ap.add_argument("--pic-steps", type=int, default=200)
    ap.add_argument("--pic-adj-steps", type=int, default=32)
    ap.add_argument("--pic-adj-every", type=int, default=16)
    ap.add_argument("--pic-adj-batch", type=int, default=50_000_000)
    ap.add_argument("--pic-warmup", type=int, default=3)
    ap.add_argument("--no-qed", action="store_true", help="skip the monopole workload (emission, conversion)")
    ap.add_argument("--qed-pairs", type=int, default=50_000_000)
    ap.add_argument("--qed-steps", type=int, default=10)
    ap.add_argument("--qed-warmup", type=int, default=3)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch

        a = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy} MiB x 5")
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs (--gpus > 1) are not supported",
              file=sys.stderr)
        sys.exit(2)

    if args.pic:
        print(json.dumps(run_pic(args, args.steps, args.warmup)), flush=True)
        return

    import torch

    from paper_2503_04558_amd import grpic

    t0 = time.time()
    g, F, parts = make_workload(args.pairs, args.nr, args.nth, args.spin, workers=args.workers)
    split_parts = None
    if not args.no_split:      # the same initial particles in split form
        split_parts = {k: (v.clone() if k in ("cell", "sp") else v.to(torch.float32)) for k, v in parts.items()}
    vay_parts = None if args.no_vay else {k: v.clone() for k, v in parts.items()}
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f}s: grid {g.nr}x{g.nth}, {2 * args.pairs} particles")
    r = run_gpu(args, g, F, parts, grpic.GRPIC_FP64)
    del parts
    rs = None
    if split_parts is not None:
        F32 = [f.to(torch.float32) for f in F]
        rs = run_gpu(args, g, F32, split_parts, grpic.GRPIC_FP32_SPLIT)
    del split_parts
    rv = None
    if vay_parts is not None:
        rv = run_gpu(args, g, F, vay_parts, grpic.GRPIC_FP64, kick="vay")
    del vay_parts
    def leg(name, skip, fn):
        """An extra leg of the bench line; a failure is reported in it and
        does not cost the line."""
        if skip:
            return None
        try:
            return fn()
        except Exception as e:                        # noqa: BLE001 -- reported in the JSON line
            log(f"{name}: failed: {e!r}")
            return {"error": repr(e)}
        finally:
            torch.cuda.empty_cache()

    fld = leg("fields", args.no_fields, lambda: run_fields(args, g, F))
    sp3 = leg("spline3", args.no_spline3, lambda: run_spline3(args))
    copy_ceiling = copy_ceiling_gbs()
    log(f"STREAM ceiling: copy {copy_ceiling['copy_gbs']} GB/s, scale {copy_ceiling['scale_gbs']} GB/s")
    adj = leg("adjoint", args.no_adjoint, lambda: run_adjoint(args))
    del F
    qed = leg("qed", args.no_qed, lambda: run_qed(args))
    pic = leg("pic", args.no_pic, lambda: run_pic(args, args.pic_steps, args.pic_warmup))
    cpu = None if args.no_cpu else run_cpu_baseline(args, g)
    # 1344 flop per 97 B = 13.9 flop/B, above the FP64 ridge (78.6 TFLOP/s / 8 TB/s =
    # 9.8 flop/B): the FP64 vector units bound this kernel, HBM comes second.
    traffic = measured_traffic()
    alu = dict(bound="alu", achieved=round(r["tflops"], 3), peak=FP64_VALU_PEAK_TFLOPS, unit="TFLOP/s",
               frac=round(r["tflops"] / FP64_VALU_PEAK_TFLOPS, 4), traffic=traffic.get("f64"),
               flops_per_launch=r["flops_per_launch"])
    hbm = dict(bound="hbm", achieved=round(r["hbm_gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(r["hbm_gbs"] / HBM_PEAK_GBS, 4), traffic=traffic.get("f64"),
               bytes_per_launch=r["bytes_per_launch"])
    out = {
        "metric": "particle push+deposit/s (FP64 vs FP32-split) at stated error; bwd/fwd time ratio",
        "value": r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["total_ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "counters": r["counters"],
        "config": {
            "workload": f"{args.nr}x{args.nth} Kerr-Schild log-r grid, a={args.spin}, Wald B0=1, "
                        f"{2 * args.pairs} e+- (Maxwell-Juttner T=0.1, 0.1c phi rotation), "
                        f"sort every {args.sort_every} steps, ncorr={args.ncorr}",
            "grid": [args.nr, args.nth], "particles": 2 * args.pairs, "spin": args.spin,
            "dt": r["dt"], "sort_every": args.sort_every, "ncorr": args.ncorr, "precision": "FP64",
        },
        "roofline": alu,
        "roofline_hbm": hbm,
        "sort_ms": r["sort_ms"],
        "sort_roofline_hbm": _sort_roofline(r["sort_ms"], 2 * args.pairs, SORT_BYTES_PER_PARTICLE_F64,
                                            measured_traffic(SORT_TRAFFIC_PROFILE, SORT_SOURCES).get("sort")),
        "hbm_copy_ceiling": copy_ceiling,
        "kernel": {"name": "push_deposit_f64_tiled", "avg_ms": r["avg_push_ms"],
                   "min_ms": float(np.min(r["push_ms"])), "bytes_per_launch": r["bytes_per_launch"],
                   "live_particles_per_launch": r["live_per_launch"]},
        "cpu_baseline": cpu,
    }
    if rs is not None:
        out["split"] = {
            "value": rs["value"], "unit": "particle-steps/s", "dtype": "f32 (f64 in r < 2M, near the axis, "
            "and for the deposit)", "ms_per_step": rs["total_ms"] / args.steps,
            "speedup_vs_fp64": rs["value"] / r["value"],
            "kernel": {"name": "push_deposit_split_tiled", "avg_ms": rs["avg_push_ms"],
                       "min_ms": float(np.min(rs["push_ms"]))},
            "roofline_hbm": dict(bound="hbm", achieved=round(rs["hbm_gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
                                 frac=round(rs["hbm_gbs"] / HBM_PEAK_GBS, 4), traffic=traffic.get("split"),
                                 bytes_per_launch=rs["bytes_per_launch"]),
            "counters": rs["counters"],
        }
    if rv is not None:
        out["vay"] = {
            "value": rv["value"], "unit": "particle-steps/s", "dtype": "f64",
            "ms_per_step": rv["total_ms"] / args.steps, "vs_boris": rv["value"] / r["value"],
            "kernel": {"name": "push_deposit_f64_tiled<kVay>", "avg_ms": rv["avg_push_ms"],
                       "min_ms": float(np.min(rv["push_ms"])), "traffic": traffic.get("vay")},
            "counters": rv["counters"],
        }
    if sp3 is not None:
        out["spline3"] = sp3
    if adj is not None:
        out["adjoint"] = adj
    if fld is not None:
        out["fields"] = fld
    if qed is not None:
        out["qed"] = qed
    if pic is not None:
        out["pic"] = pic
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
