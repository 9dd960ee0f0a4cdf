"""Benchmark of the fused finite-volume step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints ONE JSON line. The headline workload is the 4096x4096 Euler grid
(nVar = 4, Rusanov flux, transmissive boundaries, CFL 0.45, 8x8 subdomains,
seeded four-quadrant Riemann data): `value` is cell-updates per second over K
adaptive steps (each step = fluxes + update + CFL reduction of every cell),
inputs already resident in HBM. The line also carries:
  roofline     -- the fused step kernel against the 8 TB/s HBM peak, with
                  64 algorithmic bytes per cell-update (read 4 doubles, write
                  4 doubles) and the launch duration timed with HIP events on
                  the launch stream;
  cpu_baseline -- the CPU oracle on the host cores on a bounded sample;
  workloads    -- the other workloads: spray 2048^2, 256 batched grids
                  (persistent launch vs one launch per grid), the adjoint at
                  1024^2 (backward / forward cost) and advection 64^2.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LAYOUTS = {"planes": 0, "rows": 1}  # FVM_LAYOUT_PLANES, FVM_LAYOUT_ROWS
METRIC = ("Gcell-updates/s and % HBM roofline (FP64); batched vs per-grid; "
          "adjoint/forward cost")
KERNEL_SOURCES = ["fvm_kernels.hip", "fvm_step.hpp", "fvm_models.hpp", "fvm_internal.hpp"]
COUNTERS = os.path.join(ROOT, "profiles", "euler_4096_step_counters.json")
# tile shapes the autotuner measured on MI355X for these workloads (looked up
# by device, model, sizes and layout; a miss is tuned and appended)
TUNING = os.path.join(ROOT, "paper_1701_05431_amd", "tuning_mi355x.txt")


def _code_only(text: str) -> str:
    """Source text without comments and blank space: what the compiler sees
    (string literals in these files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash(read=None) -> str:
    """Hash of the step kernel's sources, comments and layout left out, so
    that counters taken on a kernel stay attached to it until its code
    changes. read(name) -> text (default: the working tree)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, "paper_1701_05431_amd", "csrc", f)) as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def timed(fn, reps: int = 1):
    """Runs fn() reps times between two HIP events on the current stream;
    returns seconds per repetition."""
    import torch
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / 1e3 / reps


def median_windows(fn, steps: int, reps: int = 5):
    """Times `reps` windows of fn() (one window = `steps` steps) with HIP
    events; returns (median ms per step, all ms per step)."""
    ms = sorted(timed(fn) / steps * 1e3 for _ in range(reps))
    return ms[len(ms) // 2], ms


def euler_protocol(s, steps: int, warmup: int, reps: int = 5, seeds=(0, 1, 2)):
    """The headline step timed as the median of `reps` windows of `steps`
    steps per seed of the Riemann data (each seed after `warmup` untimed
    steps)."""
    import torch
    from paper_1701_05431_amd import inputs
    pre = inputs.EULER_4096
    per_seed = {}
    for seed in seeds:
        s.set_state(torch.from_numpy(inputs.riemann_state(pre.nx, pre.ny, seed)))
        s.run(warmup)
        med, allv = median_windows(lambda: s.run(steps), steps, reps)
        per_seed[str(seed)] = {"median_ms_per_step": med, "ms_per_step": allv}
    meds = sorted(v["median_ms_per_step"] for v in per_seed.values())
    med = meds[len(meds) // 2]
    return {"windows_per_seed": reps, "steps_per_window": steps, "warmup_per_seed": warmup,
            "seeds": list(seeds), "per_seed": per_seed, "median_ms_per_step": med,
            "median_gcell_updates_per_s": pre.nx * pre.ny / (med * 1e-3) / 1e9,
            "median_hbm_frac": 64.0 * pre.nx * pre.ny / (med * 1e-3) / 1e9 / HBM_PEAK_GBS}


def clock_state():
    """The GPU's engine and memory clock tables and performance level from
    sysfs, when this process may read them (None otherwise)."""
    import glob
    import torch
    try:
        props = torch.cuda.get_device_properties(0)
        bus = getattr(props, "pci_bus_id", None)
        dom = getattr(props, "pci_domain_id", 0)
        dev = getattr(props, "pci_device_id", 0)
    except Exception:
        return None
    if bus is None:
        return None
    base = f"/sys/bus/pci/devices/{dom:04x}:{bus:02x}:{dev:02x}.0"
    out = {"pci": base.rsplit("/", 1)[-1]}
    for name in ("pp_dpm_sclk", "pp_dpm_mclk", "power_dpm_force_performance_level"):
        paths = glob.glob(os.path.join(base, name))
        try:
            with open(paths[0]) as fh:
                out[name] = fh.read().strip().splitlines()
        except (IndexError, OSError):
            out[name] = None
    return out


def bench_euler(args):
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.EULER_4096
    p = params_from(pre, layout=LAYOUTS[args.layout])
    s = Solver(p)
    W = inputs.riemann_state(pre.nx, pre.ny, 0)
    s.set_state(torch.from_numpy(W))
    if args.rows or args.wpb:
        s.set_tiling(args.rows, args.wpb)
    elif not args.no_autotune:
        log(f"euler: autotuned tiling (rows, waves/block, cells/lane) = {s.autotune(args.tuning)}")
    log(f"euler {pre.nx}x{pre.ny}: warmup {args.warmup}")
    s.run(args.warmup)
    torch.cuda.synchronize()
    log(f"euler: timing {args.steps} steps")
    sec = timed(lambda: s.run(args.steps))
    assert s.sync() == 0
    cells = pre.nx * pre.ny
    per_launch = sec / args.steps
    achieved = 64.0 * cells / per_launch / 1e9
    return dict(sec=sec, cells=cells, per_launch=per_launch, achieved=achieved,
                tiling=s.tiling(), cpl=s.cells_per_lane(), solver=s)


def bench_output(steps, warmup, layout="rows", tuning=TUNING):
    """Asynchronous output on the Euler 4096^2 workload: `steps` steps with
    and without a snapshot every steps/2 steps (written to the null device,
    so the disk is left out), timed on the compute stream only; and the
    gather kernel alone (one read and one write of the state)."""
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd.solver import AsyncOutput, Solver, params_from
    pre = inputs.EULER_4096
    s = Solver(params_from(pre, layout=LAYOUTS[layout]))
    s.set_state(torch.from_numpy(inputs.riemann_state(pre.nx, pre.ny, 0)))
    s.autotune(tuning)
    out = AsyncOutput(s)
    s.run(warmup)
    out.snapshot(os.devnull)
    out.wait()
    torch.cuda.synchronize()

    def compute_stream_time(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / 1e3

    plain = compute_stream_time(lambda: s.run(steps))
    half = max(1, steps // 2)

    def with_output():
        out.snapshot(os.devnull, step=0)
        s.run(half)
        out.snapshot(os.devnull, step=half)
        s.run(steps - half)

    overlapped = compute_stream_time(with_output)
    out.wait()
    torch.cuda.synchronize()
    reps = 5
    gather = []
    for _ in range(reps):
        gather.append(compute_stream_time(lambda: out.snapshot(os.devnull)))
        out.wait()
    out.close()
    st = s.sync()
    g = sorted(gather)[reps // 2]
    state_bytes = 4 * 8 * pre.nx * pre.ny
    return {"workload": pre.name, "steps": steps, "status": st, "snapshots": 2,
            "ms_plain": plain * 1e3, "ms_with_output": overlapped * 1e3,
            "overhead_frac": overlapped / plain - 1.0,
            "gather_us": g * 1e6, "gather_gbs": 2 * state_bytes / g / 1e9,
            "snapshot_bytes": state_bytes, "path": "null device"}


def bench_spray_maxent(steps, warmup, layout="rows", tuning=TUNING):
    """The spray workload with the entropy-maximising closure: a transport
    step, then the per-cell Newton source pass (FP64-bound)."""
    import torch
    from paper_1701_05431_amd import _lib, inputs
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.SPRAY_2048
    W, ug = inputs.spray_state(pre.nx, pre.ny, 0)
    s = Solver(params_from(pre, layout=LAYOUTS[layout], closure=_lib.FVM_CLOSURE_MAXENT), ug=ug)
    s.set_state(torch.from_numpy(W))
    tiling = s.autotune(tuning)
    s.run(warmup)
    cold = timed(lambda: s.run(steps))  # Newton from the normal start in every cell
    st = s.sync()
    # the same steps with every cell's multipliers kept between steps
    s.keep_closure_multipliers()
    s.set_state(torch.from_numpy(W))
    s.run(warmup)
    sec = timed(lambda: s.run(steps))
    st = st or s.sync()
    cells = pre.nx * pre.ny
    return {"workload": pre.name + "_maxent", "steps": steps, "status": st,
            "gcell_updates_per_s": cells * steps / sec / 1e9, "ms_per_step": sec / steps * 1e3,
            "newton_start": "previous step's multipliers",
            "ms_per_step_cold_start": cold / steps * 1e3,
            "tiling": {"rows_per_strip": tiling[0], "waves_per_block": tiling[1],
                       "cells_per_lane": tiling[2]}}


def bench_spray(steps, warmup, autotune=True, layout="rows", tuning=TUNING):
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.SPRAY_2048
    W, ug = inputs.spray_state(pre.nx, pre.ny, 0)
    s = Solver(params_from(pre, layout=LAYOUTS[layout]), ug=ug)
    s.set_state(torch.from_numpy(W))
    tiling = s.autotune(tuning) if autotune else s.tiling() + (s.cells_per_lane(),)
    s.run(warmup)
    sec = timed(lambda: s.run(steps))
    st = s.sync()
    per = sec / steps
    cells = pre.nx * pre.ny
    gbs = 112.0 * cells / per / 1e9
    return {"workload": pre.name, "steps": steps, "status": st,
            "gcell_updates_per_s": cells * steps / sec / 1e9, "ms_per_step": per * 1e3,
            "bytes_per_cell": 112, "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "tiling": {"rows_per_strip": tiling[0], "waves_per_block": tiling[1],
                       "cells_per_lane": tiling[2]}}


def bench_batch(steps, warmup, layout="rows", tuning=TUNING):
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd.solver import Batch, aligned_pitch, params_from
    sizes = inputs.batch_sizes(inputs.BATCH_COUNT, 0)
    # pitches rounded up to 128 bytes: rows start on cache lines
    plist = [params_from(inputs.BATCH_256, nx=n, ny=n, ld=aligned_pitch(n),
                         layout=LAYOUTS[layout])
             for n in sizes]
    states = [inputs.riemann_state(n, n, k) for k, n in enumerate(sizes)]
    cells = sum(n * n for n in sizes)
    out = {"workload": inputs.BATCH_256.name, "grids": len(sizes), "cells": cells,
           "pitch": "nx rounded up to a multiple of 16 doubles",
           "steps": steps}
    for name, per_grid in (("persistent", False), ("per_grid", True)):
        b = Batch(plist)
        b.set_states(states)
        if per_grid:
            # the reference schedule gets its best tile shape too
            cands = [(8, 1), (16, 2), (32, 4), (64, 8)]
        else:
            b.autotune(tuning)
            cands = [None]
        best = None
        for c in cands:
            if c:
                b.set_tiling(*c)
            b.set_states(states)
            b.run(warmup, per_grid=per_grid)
            sec = timed(lambda: b.run(steps, per_grid=per_grid))
            if best is None or sec < best[0]:
                best = (sec, c)
        sec = best[0]
        st = b.sync()
        gbs = 64.0 * cells * steps / sec / 1e9
        out[name] = {"gcell_updates_per_s": cells * steps / sec / 1e9,
                     "ms_per_step": sec / steps * 1e3, "hbm_frac": gbs / HBM_PEAK_GBS,
                     "status": st}
        del b
    out["batched_vs_per_grid"] = (out["persistent"]["gcell_updates_per_s"] /
                                  out["per_grid"]["gcell_updates_per_s"])
    return out


def bench_adjoint(reps, layout="rows", tuning=TUNING):
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.ADJOINT_1024
    every = inputs.ADJOINT_CKPT_EVERY
    W = inputs.riemann_state(pre.nx, pre.ny, 0)
    tgt = torch.from_numpy(inputs.adjoint_target_density(pre.nx, pre.ny, 0)).cuda()
    s = Solver(params_from(pre, layout=LAYOUTS[layout]))
    Wt = torch.from_numpy(W).cuda()
    s.set_state(Wt)
    s.autotune(tuning)
    # the adjoint's tiles, timed on multiplier buffers like the backward pass's
    la = s._as_state(torch.zeros((s.nv, pre.ny, pre.nx), dtype=torch.float64))
    s.autotune_adjoint(s._as_state(Wt), la, torch.empty_like(la), tuning)
    holder = {}

    def fwd():
        s.set_state(Wt)
        holder["ck"], holder["dts"] = s.run_ckpt(pre.nsteps, every)

    def bwd():
        cur = s.current()[:, :, :pre.nx]
        lam = torch.zeros((s.nv, pre.ny, pre.nx), dtype=torch.float64, device="cuda")
        lam[0] = cur[0] - tgt
        holder["g"] = s.adjoint(holder["ck"], every, holder["dts"], lam)

    fwd()
    bwd()
    tf = min(timed(fwd) for _ in range(reps))
    fwd()
    tb = min(timed(bwd) for _ in range(reps))
    cells = pre.nx * pre.ny
    return {"workload": pre.name, "steps": pre.nsteps, "ckpt_every": every,
            "forward_ms": tf * 1e3, "backward_ms": tb * 1e3,
            "adjoint_over_forward": tb / tf,
            "forward_gcell_updates_per_s": cells * pre.nsteps / tf / 1e9,
            "status": s.sync()}


def bench_adjoint_step_4096(reps, layout="rows", tuning=TUNING):
    """One adjoint step of the 4096^2 Euler grid (reads W^n and lam^{n+1},
    writes lam^n: 96 algorithmic bytes per cell), timed per launch."""
    import ctypes as C
    import torch
    import numpy as np
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd._lib import check, lib
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.EULER_4096
    s = Solver(params_from(pre, layout=LAYOUTS[layout]))
    W0 = torch.from_numpy(inputs.riemann_state(pre.nx, pre.ny, 0))
    W = s._as_state(W0)  # storage in the grid's layout
    g = torch.Generator().manual_seed(0)
    la = s._as_state(torch.randn((s.nv, pre.ny, pre.nx), dtype=torch.float64, generator=g))
    lb = torch.empty_like(la)
    s.set_state(W0)
    s.autotune(tuning)
    s.autotune_adjoint(W, la, lb, tuning)  # the adjoint's tiles, on these buffers
    dt = s.cfl_dt()[0]
    L = lib()
    ptr = lambda t: C.c_void_p(t.data_ptr())
    s._bind_stream()

    def two():
        check(L.fvm_adjoint_step(s.h, ptr(W), dt, ptr(la), ptr(lb)), "fvm_adjoint_step")
        check(L.fvm_adjoint_step(s.h, ptr(W), dt, ptr(lb), ptr(la)), "fvm_adjoint_step")

    two()
    sec = timed(two, reps) / 2
    assert bool(torch.isfinite(la).all())
    cells = pre.nx * pre.ny
    gbs = 96.0 * cells / sec / 1e9
    return {"workload": "euler_adjoint_step_4096x4096", "us_per_step": sec * 1e6,
            "bytes_per_cell": 96, "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "gcell_updates_per_s": cells / sec / 1e9}


def bench_spray_adjoint(reps, steps=20, layout="rows", tuning=TUNING):
    """The spray's discrete adjoint on the 2048^2 spray workload (lognormal
    closure): one adjoint step timed per launch (reads W^n, lam^{n+1} and the
    gas velocity, writes lam^n: 160 algorithmic bytes per cell), and a
    checkpointed differentiable run of `steps` steps against its forward."""
    import ctypes as C
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd._lib import check, lib
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.SPRAY_2048
    W0, ug = inputs.spray_state(pre.nx, pre.ny, 0)
    s = Solver(params_from(pre, layout=LAYOUTS[layout]), ug=ug)
    W0 = torch.from_numpy(W0)
    W = s._as_state(W0)
    g = torch.Generator().manual_seed(0)
    la = s._as_state(torch.randn((s.nv, pre.ny, pre.nx), dtype=torch.float64, generator=g))
    lb = torch.empty_like(la)
    s.set_state(W0)
    s.autotune(tuning)
    dt = s.cfl_dt()[0]
    L = lib()
    ptr = lambda t: C.c_void_p(t.data_ptr())
    s._bind_stream()

    def two():
        check(L.fvm_adjoint_step(s.h, ptr(W), dt, ptr(la), ptr(lb)), "fvm_adjoint_step")
        check(L.fvm_adjoint_step(s.h, ptr(W), dt, ptr(lb), ptr(la)), "fvm_adjoint_step")

    two()
    sec = timed(two, reps) / 2
    assert bool(torch.isfinite(la).all())
    cells = pre.nx * pre.ny
    gbs = 160.0 * cells / sec / 1e9
    every = 5
    holder = {}
    W0d = W0.cuda()

    def fwd():
        s.set_state(W0d)
        holder["ck"], holder["dts"] = s.run_ckpt(steps, every)

    def bwd():
        lam = s.current()[:, :, :pre.nx].clone()
        holder["g"] = s.adjoint(holder["ck"], every, holder["dts"], lam)

    fwd()
    bwd()
    tf = min(timed(fwd) for _ in range(3))
    fwd()
    tb = min(timed(bwd) for _ in range(3))
    return {"workload": "spray_adjoint_2048x2048", "us_per_step": sec * 1e6,
            "bytes_per_cell": 160, "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "gcell_updates_per_s": cells / sec / 1e9, "run_steps": steps,
            "ckpt_every": every, "forward_ms": tf * 1e3, "backward_ms": tb * 1e3,
            "adjoint_over_forward": tb / tf, "status": s.sync()}


def bench_slab(steps, warmup, layout="rows", tuning=TUNING):
    """One GPU's share of the 4096^2 Euler grid cut into 8 slabs of 512 rows:
    the slab steps with its south and north halo rows read from neighbour
    buffers (the rows an exchange between GPUs would deliver)."""
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.EULER_4096
    rows = pre.ny // 8
    W = inputs.riemann_state(pre.nx, pre.ny, 0)
    q = 3  # a slab in the middle of the grid
    s = Solver(params_from(pre, ny=rows, npart_y=1, ly=rows / pre.ny, layout=LAYOUTS[layout]))
    s.set_state(torch.from_numpy(W[:, q * rows:(q + 1) * rows]))
    s.autotune(tuning)
    south = torch.from_numpy(W[:, q * rows - 1, :].copy()).cuda().contiguous()
    north = torch.from_numpy(W[:, (q + 1) * rows, :].copy()).cuda().contiguous()
    s.set_halo_rows(south, north)
    s.run(warmup)
    sec = timed(lambda: s.run(steps))
    cells = pre.nx * rows
    per = sec / steps
    gbs = 64.0 * cells / per / 1e9
    return {"workload": "euler_slab_4096x512_halo_rows", "steps": steps, "status": s.sync(),
            "us_per_step": per * 1e6, "gcell_updates_per_s": cells / per / 1e9,
            "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "halo_bytes_per_step": 2 * 4 * pre.nx * 8,
            "tiling": {"rows_per_strip": s.tiling()[0], "waves_per_block": s.tiling()[1],
                       "cells_per_lane": s.cells_per_lane()}}


def bench_advection(steps):
    import torch
    from paper_1701_05431_amd import inputs
    from paper_1701_05431_amd.solver import Solver, params_from
    pre = inputs.ADVECTION_64
    s = Solver(params_from(pre))
    s.set_state(torch.from_numpy(inputs.advection_state(64, 64, 0)))
    s.run(pre.nsteps)
    sec = timed(lambda: s.run(pre.nsteps), reps=5)
    return {"workload": pre.name, "steps": pre.nsteps, "us_per_step": sec / pre.nsteps * 1e6,
            "status": s.sync()}


def cpu_share() -> tuple[int, int]:
    """(threads the CPU baseline uses, host cores visible to this process):
    one GPU's share of a shared host is 16 cores, whatever the affinity
    mask shows."""
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    return min(visible, 16), visible


def _oracle_step_cost(run, k_target_s: float):
    """Per-step seconds of an oracle run(n) call, from a one-step and a
    three-step call (a call has a fixed cost, the subdomain copies in and
    out, besides its steps); returns (per_step, t1, t3)."""
    t0 = time.perf_counter()
    run(1)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    run(3)
    t3 = time.perf_counter() - t0
    return max((t3 - t1) / 2.0, 1e-4), t1, t3


def cpu_baseline(target_s: float = 10.0):
    """The oracle as it is, on the host: the headline Euler workload on the
    CPU share (value) and on one core, bounded samples of the spray and
    batch workloads, and the oracle's adjoint at 256^2; per-step times are
    extrapolated to each workload's step count."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import fv as orc
    from paper_1701_05431_amd import inputs
    cores, visible = cpu_share()
    pre = inputs.EULER_4096
    cells = pre.nx * pre.ny
    orc.set_threads(cores)
    P = orc.from_preset(pre)
    W = inputs.riemann_state(pre.nx, pre.ny, 0)
    W, _ = orc.run(P, W, 1)  # warm-up: thread start-up, first touch of the arrays
    per, t1, _ = _oracle_step_cost(lambda n: orc.run(P, W, n), target_s)
    k = max(1, min(1000, int((target_s - max(t1 - per, 0.0)) / per)))
    t0 = time.perf_counter()
    orc.run(P, W, k)
    t = time.perf_counter() - t0
    value = cells * k / t / 1e9
    # one core: the per-step cost from a one- and a three-step call
    orc.set_threads(1)
    per1, _, _ = _oracle_step_cost(lambda n: orc.run(P, W, n), target_s)
    one_core = {"cores": 1, "gcell_updates_per_s": cells / per1 / 1e9, "s_per_step": per1,
                "extrapolated_s_200_steps": 200 * per1,
                "sample": f"{pre.name}: (three-step call - one-step call) / 2, one thread"}
    # spray workload
    sp = inputs.SPRAY_2048
    Ps = orc.from_preset(sp)
    Ws, ug = inputs.spray_state(sp.nx, sp.ny, 0)
    spray = {}
    for nthr in (cores, 1):
        orc.set_threads(nthr)
        ps, _, _ = _oracle_step_cost(lambda n: orc.run(Ps, Ws, n, ug), target_s)
        spray[str(nthr)] = {"cores": nthr, "gcell_updates_per_s": sp.nx * sp.ny / ps / 1e9,
                            "s_per_step": ps, "extrapolated_s_200_steps": 200 * ps}
    # batch workload: every grid, one call per grid, grids spread over the
    # share's threads (one thread per call: the grids have one subdomain)
    sizes = inputs.batch_sizes(inputs.BATCH_COUNT, 0)
    bcells = sum(n * n for n in sizes)
    bstates = [inputs.riemann_state(n, n, g) for g, n in enumerate(sizes)]

    def grid_cost(gn):
        g, n = gn
        orc.set_threads(1)
        Pg = orc.from_preset(inputs.BATCH_256, nx=n, ny=n, npx=1, npy=1)
        t0 = time.perf_counter()
        orc.run(Pg, bstates[g], 1)
        a = time.perf_counter() - t0
        t0 = time.perf_counter()
        orc.run(Pg, bstates[g], 3)
        return (time.perf_counter() - t0 - a) / 2.0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        costs = list(ex.map(grid_cost, list(enumerate(sizes))))
    wall = time.perf_counter() - t0
    step_1core = sum(costs)
    batch = {"grids": len(sizes), "cells": bcells, "threads": cores,
             "s_per_step_one_core": step_1core,
             "gcell_updates_per_s_one_core": bcells / step_1core / 1e9,
             "s_per_step_share": step_1core / cores,
             "gcell_updates_per_s_share": bcells / (step_1core / cores) / 1e9,
             "extrapolated_s_100_steps_share": 100 * step_1core / cores,
             "sample": "each grid's (three-step call - one-step call) / 2 on one thread, "
                       f"grids spread over {cores} threads ({wall:.1f} s wall); the share's rate "
                       "assumes the grids divide evenly over its threads"}
    # the oracle's adjoint (one thread) on the adjoint workload's kind of
    # state at 256^2: forward states kept, then the adjoint steps
    adj = inputs.ADJOINT_1024
    n, steps = 256, 10
    Pa = orc.from_preset(adj, nx=n, ny=n, npx=1, npy=1)
    Wa = inputs.riemann_state(n, n, 0)
    _, dts = orc.run(Pa, Wa, steps)
    lam = np.zeros_like(Wa)
    lam[0] = 1.0
    t0 = time.perf_counter()
    orc.adjoint_run(Pa, Wa, dts, lam)
    ta = time.perf_counter() - t0
    orc.set_threads(cores)
    return {"value": value, "unit": "Gcell-updates/s", "cores": cores, "kind": "oracle",
            "host_cores_visible": visible,
            "sample": f"{pre.name}: {k} adaptive steps in one call ({t:.1f} s) after 5 "
                      f"untimed steps, {cores} threads (one GPU's share of the host)",
            "extrapolated_s_200_steps": 200 * t / k,
            "one_core": one_core, "spray": spray, "batch": batch,
            "adjoint": {"workload": f"euler_adjoint_{n}x{n}", "steps": steps, "cores": 1,
                        "ms_per_step": ta / steps * 1e3,
                        "sample": "forward states recomputed and kept, then the adjoint "
                                  "steps, one call"}}


def traffic_from_counters(tiling: dict, layout: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel source in the same launch
    configuration."""
    if not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as fh:
        c = json.load(fh)
    if c.get("kernel_hash") != kernel_hash() or c.get("tiling") != tiling:
        return None
    if c.get("layout") != layout:
        return None
    return c.get("bytes_per_launch")


def copy_probe(nbytes: int, reps: int):
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--wpb", type=int, default=0)
    ap.add_argument("--only-euler", action="store_true")
    ap.add_argument("--only", choices=["spray", "batch", "adjoint", "adjoint4096", "slab",
                                       "advection", "output", "spray_maxent",
                                       "spray_adjoint"],
                    help="run just this secondary workload (for profiling) and print its record")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default=TUNING,
                    help="autotuner cache file (tile shapes measured on this device)")
    ap.add_argument("--layout", choices=sorted(LAYOUTS), default="rows",
                    help="state storage: one plane per variable, or the variables' rows "
                         "interleaved per grid row")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, help="bytes of a plain D2D copy")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the finite-volume path here runs on a single "
              "MI355X; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe, 10)
        return
    if args.only:
        run = {"adjoint4096": lambda: bench_adjoint_step_4096(50, args.layout, args.tuning),
               "slab": lambda: bench_slab(args.steps, args.warmup, args.layout, args.tuning),
               "spray": lambda: bench_spray(args.steps, args.warmup, not args.no_autotune,
                                            args.layout, args.tuning),
               "batch": lambda: bench_batch(args.steps, args.warmup, args.layout, args.tuning),
               "adjoint": lambda: bench_adjoint(1, args.layout, args.tuning),
               "advection": lambda: bench_advection(args.steps),
               "output": lambda: bench_output(args.steps, args.warmup, args.layout,
                                              args.tuning),
               "spray_maxent": lambda: bench_spray_maxent(min(args.steps, 20), 2, args.layout,
                                                          args.tuning),
               "spray_adjoint": lambda: bench_spray_adjoint(20, 20, args.layout,
                                                            args.tuning)}[args.only]
        print(json.dumps(run()), flush=True)
        return

    e = bench_euler(args)
    value = e["cells"] * args.steps / e["sec"] / 1e9
    log("euler: median of 5 windows for seeds 0, 1, 2")
    protocol = euler_protocol(e["solver"], args.steps, args.warmup)
    protocol["clock_state"] = clock_state()
    tiling = {"rows_per_strip": e["tiling"][0], "waves_per_block": e["tiling"][1],
              "cells_per_lane": e["cpl"]}
    traffic = traffic_from_counters(tiling, args.layout)
    roof = {"bound": "hbm", "achieved": e["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": e["achieved"] / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "fvm::step_kernel<Euler, transmissive>",
            "algorithmic_bytes_per_launch": 64 * e["cells"],
            "avg_launch_ms": e["per_launch"] * 1e3}
    del e["solver"]
    work = {}
    if not args.only_euler:
        log("spray")
        work["spray"] = bench_spray(200, 10, layout=args.layout, tuning=args.tuning)
        log("batch")
        work["batch"] = bench_batch(100, 4, args.layout, args.tuning)
        log("adjoint")
        work["adjoint"] = bench_adjoint(3, args.layout, args.tuning)
        log("adjoint step 4096")
        work["adjoint_step_4096"] = bench_adjoint_step_4096(50, args.layout, args.tuning)
        log("spray adjoint")
        work["spray_adjoint"] = bench_spray_adjoint(20, 20, args.layout, args.tuning)
        log("slab with halo rows")
        work["slab"] = bench_slab(200, 20, args.layout, args.tuning)
        log("advection")
        work["advection"] = bench_advection(100)
        log("spray, entropy-maximising closure")
        work["spray_maxent"] = bench_spray_maxent(20, 2, args.layout, args.tuning)
        log("asynchronous output")
        work["output"] = bench_output(200, 20, args.layout, args.tuning)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": e["sec"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "euler_4096x4096", "nx": 4096, "ny": 4096, "nvar": 4,
                   "flux": "rusanov", "bc": "transmissive", "cfl": 0.45, "subdomains": "8x8",
                   "init": "four-quadrant Riemann, seed 0", "layout": args.layout,
                   "tiling": tiling},
        "roofline": roof,
        "timing_protocol": protocol,
        "cpu_baseline": cpu,
        "workloads": work,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
