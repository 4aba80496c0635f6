"""Benchmark: WCSPH dam-break step throughput on one MI355X.

Workload (default): the 3-D dam break with 1,000,000 fluid particles
(dp = 0.002 m, 0.2 m cube against the corner of a 0.8 x 0.4 x 0.4 m open tank)
plus 648,032 dynamic boundary particles, FP32 pair arithmetic, cell list
rebuilt every step.  One step = sph_build_cells -> sph_interact -> sph_step
(neighbour list, particle interaction, Verlet update with CFL time step).

Prints ONE JSON line.  ``value`` is directed pair interactions per second over
the K timed steps (inputs resident in HBM, no host transfer inside the timed
region).  ``roofline`` reports the pair kernel (one fused launch per step:
fluid targets, then boundary targets; the dominant kernel) against the FP32
vector ALU peak; ``cpu_baseline`` times the FP64
oracle on the host cores on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair interactions/s + steps/s, 1M-particle dam break FP32; adjoint/forward time"
# Algorithmic FP32 operations per directed pair (FMA = 2), counted from the
# pair arithmetic of the method: a fluid target costs r and r^2 8, sqrt 1,
# kernel gradient factor 5, v_ab and v.r 8, continuity 2, mu 4, max |mu| 1,
# rho_b and c_b 5, Monaghan term 6, pressure terms 2, coefficient 1,
# momentum 6 (49); a boundary target only the distance, kernel factor, v.r
# and continuity terms (24).
FLOP_FLUID_PAIR = 49
FLOP_BOUND_PAIR = 24
# the cubic spline's gradient factor costs one operation more than the
# Wendland one; the tensile correction adds 13 per fluid-target pair (kernel
# shape 6, f^4 2, R_b 2, R_ab 1, accumulate 2)
FLOP_CUBIC_EXTRA = 1
FLOP_TENSILE_EXTRA = 13
PEAK_FP32_VECTOR = 157.3e12   # MI355X FP32 vector peak (FLOP/s)
PAPER_CONTEXT = "GTX 480: 10.1 steps/s at 1,011,354 particles (paper Table 4; other hardware, " \
                "cubic-spline kernel, own geometry)"


def _kernel_source_hash():
    p = os.path.join(ROOT, "paper_1110_3711_amd", "csrc", "interact.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def _traffic_record():
    """HBM bytes per launch of the fused pair kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "interact_dam_break_1m_traffic.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("kernel_source_sha256_16") != _kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def _host_cpu():
    """CPU model name (from /proc/cpuinfo) and the logical CPUs this process
    may run on."""
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        nproc = os.cpu_count()
    return model, nproc


def cpu_baseline(layout, budget_s: float = 12.0):
    """Time the FP64 oracle (as it stands) on the host cores: whole steps
    (interact + time step + Verlet) of the same layout."""
    import oracle

    S = oracle.State(layout)
    # pairs per step from one untimed interact on the initial state
    _, _, nnb, npairs = S.interact()
    t0 = time.perf_counter()
    steps = 0
    while True:
        S.run(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 20:
            break
    dt = time.perf_counter() - t0
    model, nproc = _host_cpu()
    return {
        "value": npairs * steps / dt,
        "unit": "pair interactions/s",
        "steps_per_s": steps / dt,
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} whole FP64 steps (cell list, OpenMP over targets) of the same "
                  f"{layout.n:,}-particle layout; pairs/step {npairs:,} from the initial state",
        "cpu": model,
        "nproc": nproc,
    }


def adjoint_ratio(layout, steps: int, every: int, reps: int = 3):
    """Wall time of the checkpointed backward pass (recompute + adjoint) over
    the forward pass of the same rollout (both on the device, synchronised),
    median over `reps` repetitions (small layouts are partly bound by host
    launch overhead, which varies from run to run), and the peak device
    memory."""
    import torch

    from paper_1110_3711_amd.rollout import Rollout

    torch.cuda.reset_peak_memory_stats()
    roll = Rollout(layout, steps, every)
    v0 = torch.as_tensor(layout.v[layout.nb:], dtype=torch.float64, device=roll.device)
    rng = np.random.default_rng(7)
    target = torch.as_tensor(layout.x[layout.nb:].mean(0) + rng.uniform(-0.01, 0.01, 3),
                             device=roll.device)
    # untimed warm-up of every kernel on a short rollout
    warm = Rollout(layout, every, every)
    xw = warm.forward(layout.phys.alpha, v0)
    warm.backward(torch.ones_like(xw))
    del warm
    runs = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xk = roll.forward(layout.phys.alpha, v0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gx = 2.0 / 3.0 * (xk.mean(0) - target) / xk.shape[0]
        ga, gv = roll.backward(gx.expand_as(xk).contiguous())
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        runs.append((t1 - t0, t2 - t1))
    ratios = [b / f for f, b in runs]
    k = int(np.argsort(ratios)[len(ratios) // 2])
    ok = bool(torch.isfinite(gv).all().item()) and bool(torch.isfinite(ga).item())
    return {"workload": layout.name, "particles": layout.n, "ratio": ratios[k],
            "ratios": ratios, "forward_s": runs[k][0], "backward_s": runs[k][1],
            "steps": steps, "checkpoint_every": every, "finite": ok,
            "alpha_grad": float(ga.item()),
            "peak_device_bytes": int(torch.cuda.max_memory_allocated())}


def timed_steps(sim, K: int, warmup: int):
    """Warm up, then time K whole steps (build_cells -> interact -> update) on
    the current stream: HIP events around every pair stage and, on every 8th
    step, around the whole step; inputs stay in HBM throughout."""
    import torch

    from paper_1110_3711_amd import sph

    stream = torch.cuda.current_stream()
    # warmup (also brings the dam-break state past its first steps)
    for _ in range(warmup):
        sim.step()
    torch.cuda.synchronize()
    if sim.dev_status() & sph.SPH_DEV_NONFINITE:
        raise SystemExit("non-finite state during warmup")
    npairs = torch.zeros(2, dtype=torch.int64, device=sim.device)  # fluid, boundary targets
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    # per-stage events of every 8th step (before the neighbour list, after the
    # update): sampled, so that the extra event records barely touch the timing
    SAMPLE = 8
    es = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in range(0, K, SAMPLE)}
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    t0 = time.perf_counter()
    for k in range(K):
        if k in es:
            es[k][0].record(stream)
        sim.build_cells()
        ev[k][0].record(stream)
        sim.interact(parts=sph.SPH_PI_ALL, npairs=npairs)
        ev[k][1].record(stream)
        sim.update()
        if k in es:
            es[k][1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = sim.check_status()
    if status & sph.SPH_DEV_NONFINITE:
        raise SystemExit("non-finite state in the timed region")
    return {
        "gpu_ms": start.elapsed_time(stop),
        "wall": wall,
        "status": status,
        "pi_ms": np.array([a.elapsed_time(b) for a, b in ev]),
        "nl_ms": np.array([es[k][0].elapsed_time(ev[k][0]) for k in es]),
        "su_ms": np.array([ev[k][1].elapsed_time(es[k][1]) for k in es]),
        "pf": int(npairs[0].item()),
        "pb": int(npairs[1].item()),
    }


def large_leg(config: str, steps: int, warmup: int):
    """A few timed steps of the largest single-GPU layout: throughput, pair
    kernel rate against the FP32 peak, peak device memory."""
    import torch

    from paper_1110_3711_amd import sph
    from sph_inputs import CASES, named_case

    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    lay = named_case(config)
    sim = sph.Simulation(lay, nsub=1)
    R = timed_steps(sim, steps, warmup)
    pairs = R["pf"] + R["pb"]
    t = R["gpu_ms"] / 1e3
    flop_launch = (R["pf"] * FLOP_FLUID_PAIR + R["pb"] * FLOP_BOUND_PAIR) / steps
    achieved = flop_launch / (R["pi_ms"].mean() / 1e3)
    out = {
        "workload": f"{config}: {CASES[config].description}",
        "particles": lay.n,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": R["gpu_ms"] / steps,
        "steps_per_s": steps / t,
        "pairs_per_s": pairs / t,
        "pairs_per_step": pairs / steps,
        "stage_ms": {"build_cells": float(R["nl_ms"].mean()), "interact": float(R["pi_ms"].mean()),
                     "step": float(R["su_ms"].mean())},
        "pair_kernel_tflops": achieved / 1e12,
        "pair_kernel_frac": achieved / PEAK_FP32_VECTOR,
        "peak_device_bytes": int(torch.cuda.max_memory_allocated()),
        "dev_status": R["status"],
    }
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="dam_break_1m")
    ap.add_argument("--nsub", type=int, default=1)
    ap.add_argument("--kernel", choices=["wendland", "cubic"], default="wendland",
                    help="smoothing kernel (cubic: the Table 1 spline, with alpha = 0.25)")
    ap.add_argument("--tensile", action="store_true",
                    help="tensile correction on (spacing = the layout's dp)")
    ap.add_argument("--range-table", action="store_true",
                    help="precomputed interaction ranges per cell (Section 4.4, optimisation D)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--adjoint-config", default="dam_break_64k",
                    help="layout of the differentiable rollout (default: the 64k-fluid case)")
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--adjoint-every", type=int, default=20)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--large-config", default="dam_break_20m",
                    help="layout of the large single-GPU leg (a few timed steps)")
    ap.add_argument("--large-steps", type=int, default=10)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); the "
              "multi-GPU slab decomposition is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1110_3711_amd import sph
    from sph_inputs import CASES, named_case

    if args.calibrate_copy:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    def variant(layout):
        if args.kernel == "cubic":
            layout.phys = dataclasses.replace(layout.phys, kernel=1, alpha=0.25)
        if args.tensile:
            layout.phys = dataclasses.replace(layout.phys, tensile_dp=layout.phys.dp)
        return layout

    lay = variant(named_case(args.config))
    torch.cuda.reset_peak_memory_stats()
    sim = sph.Simulation(lay, nsub=args.nsub, ranges=args.range_table)
    R = timed_steps(sim, args.steps, args.warmup)
    K = args.steps
    pf, pb, pi_ms, nl_ms, su_ms = R["pf"], R["pb"], R["pi_ms"], R["nl_ms"], R["su_ms"]
    pairs = pf + pb
    gpu_ms, wall, status = R["gpu_ms"], R["wall"], R["status"]
    t = gpu_ms / 1e3
    ms_step = gpu_ms / K

    # one fused pair-kernel launch per step: fluid targets (F-F + F-B), then
    # boundary targets (B-F)
    ffl = FLOP_FLUID_PAIR + (FLOP_CUBIC_EXTRA if args.kernel == "cubic" else 0) + \
        (FLOP_TENSILE_EXTRA if args.tensile else 0)
    fbd = FLOP_BOUND_PAIR + (FLOP_CUBIC_EXTRA if args.kernel == "cubic" else 0)
    flop_launch = (pf * ffl + pb * fbd) / K
    # the committed counter record holds the default kernel (Wendland, no
    # tensile correction) on the 1M-particle layout only
    default_path = (args.config == "dam_break_1m" and args.kernel == "wendland" and
                    not args.tensile and args.nsub == 1 and not args.range_table)
    traffic = _traffic_record() if default_path else None
    achieved = flop_launch / (pi_ms.mean() / 1e3)
    roof = {
        "bound": "alu",
        "kernel": "k_interact<fused> (fluid targets F-F + F-B, then boundary targets B-F)",
        "achieved": achieved / 1e12,
        "peak": PEAK_FP32_VECTOR / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_VECTOR,
        "traffic": traffic,
        "traffic_GBps": None if traffic is None else traffic / (pi_ms.mean() / 1e3) / 1e9,
        "avg_launch_ms": float(pi_ms.mean()),
        "pairs_per_launch": (pf + pb) / K,
        "fluid_target_pairs_per_launch": pf / K,
        "boundary_target_pairs_per_launch": pb / K,
        "flop_per_pair": {"fluid_target": ffl, "boundary_target": fbd},
    }

    out = {
        "metric": METRIC,
        "value": pairs / t,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: {CASES[args.config].description}",
            "particles": lay.n,
            "fluid": lay.nf,
            "boundary": lay.nb,
            "nsub": args.nsub,
            "cells": sim.ncell,
            "range_table": bool(args.range_table),
            "kernel": ("cubic spline, alpha = 0.25" if args.kernel == "cubic" else
                       "Wendland quintic") + ", h = 1.2 sqrt(3) dp, support 2h" +
                      (", tensile correction" if args.tensile else ""),
            "parallelism": "single GPU",
        },
        "steps_per_s": K / t,
        # mean per-step time of each stage from HIP events inside the timed region
        # (neighbour list and update on every 8th step, interaction on every step)
        "stage_ms": {"build_cells": float(nl_ms.mean()), "interact": float(pi_ms.mean()),
                     "step": float(su_ms.mean())},
        # every unordered F-F or F-B pair is evaluated from both of its ends
        "unordered_pairs_per_s": pairs / 2 / t,
        "pairs_per_step": pairs / K,
        "wall_s": wall,
        "adjoint_forward_ratio": None,
        "adjoint": None,
        "dev_status": status,
        "peak_device_bytes": int(torch.cuda.max_memory_allocated()),
        "paper_context": PAPER_CONTEXT,
        "roofline": roof,
    }
    del sim
    torch.cuda.empty_cache()
    if not args.no_large:
        out["large"] = large_leg(args.large_config, args.large_steps, 3)
    if not args.no_adjoint:
        alay = lay if args.adjoint_config == args.config else variant(named_case(args.adjoint_config))
        adj = adjoint_ratio(alay, args.adjoint_steps, args.adjoint_every)
        out["adjoint"] = adj
        out["adjoint_forward_ratio"] = adj["ratio"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lay, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
