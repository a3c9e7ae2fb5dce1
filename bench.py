#!/usr/bin/env python3
"""Throughput of the compressed particle-mesh step (1-byte positions and velocities) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3_pm2048]

One step = the whole hot path on the resident compressed state: integer CIC deposit, five-pass
FFT Poisson solve, force interpolation + kick + drift + re-encode (count pass, per-cell link and
scan, scatter pass). Initial conditions are generated on the GPU before the timed region.
Prints one JSON line: particle-steps/s, the roofline of the dominant kernel (algorithmic bytes
per launch over its HIP-event-timed duration, against the 8 TB/s HBM peak) and the oracle timed
on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNELS = ("deposit", "fft_x", "fft_y", "fft_z_green", "fft_y_inv", "fft_x_inv", "move_count", "link_scan",
           "move_scatter")


def algorithmic_bytes(cfg: dict) -> dict:
    """Minimal HBM bytes per launch of each kernel (they add up to the step's algorithmic bytes):
    particle streams 3 n_chi (deposit read), 3 (n_chi + n_nu) (move read), 3 (n_chi + n_nu)
    (encode write) per particle; 4 bytes per fine cell for the density write and the potential
    read, 8 per fine cell for each FFT pass (read + write of the half spectrum); 24 bytes per
    coarse cell read (offset, mean velocity, scale) and 24 written."""
    n = cfg["np_side"] ** 3
    nm3 = cfg["nm_side"] ** 3
    nc3 = cfg["nc_side"] ** 3
    x, v = cfg["x_bytes"], cfg["v_bytes"]
    fft = 8.0 * nm3
    return {
        "deposit": 3.0 * x * n + 4.0 * nm3,
        "fft_x": fft, "fft_y": fft, "fft_z_green": fft, "fft_y_inv": fft, "fft_x_inv": fft,
        "move_count": 3.0 * (x + v) * n + 4.0 * nm3 + 24.0 * nc3,
        "link_scan": 24.0 * nc3,
        "move_scatter": 3.0 * (x + v) * n,
    }


def cpu_baseline(cfg: dict, sample_side: int, steps: int):
    """The oracle (plain FP64 numpy PM on uncompressed particles) on a sub-box with the workload's
    particle and mesh resolution; particle-steps per second of host time."""
    import numpy as np
    from oracle import ic, pm
    from oracle.cosmology import Cosmology

    ratio = cfg["nm_side"] // cfg["np_side"]
    nm = sample_side * ratio
    box = cfg["box"] * sample_side / cfg["np_side"]
    cosmo = Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])
    x, p, _ = ic.zeldovich(sample_side, nm, box, cosmo, cfg["a_init"], cfg["seed"])
    run = pm.PMRun(x, p, nm, cosmo, cfg["a_init"], cfg["a_final"], cfg["n_steps"], cfg.get("spacing", 0))
    run.advance()  # initial half drift, untimed
    t0 = time.perf_counter()
    for _ in range(steps):
        run.advance()
    dt = time.perf_counter() - t0
    n = sample_side**3
    return {
        "value": n * steps / dt,
        "unit": "particle-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} DKD steps of the FP64 numpy oracle on a {sample_side}^3-particle, {nm}^3-mesh "
                  f"sub-box ({box:g} Mpc/h, same particle and mesh resolution as the workload); "
                  f"{dt:.1f} s on 1 host thread (numpy FFT and bincount are single-threaded)",
        "seconds": dt,
        "host_cpus": os.cpu_count(),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3_pm2048", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--cpu-sample-side", type=int, default=128)
    ap.add_argument("--cpu-sample-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (one box per GPU; "
              "the sharded design is described in DESIGN.md). Use --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from paper_1712_06121_amd import SIGMA_PER_CELL, Sim

    torch.cuda.set_device(0)
    cfg = dict(synth.WORKLOADS[args.workload])
    if args.warmup + args.steps > cfg["n_steps"]:
        print(f"warmup + steps must not exceed the schedule's {cfg['n_steps']} steps", file=sys.stderr)
        return 2
    print(f"[bench] workload {args.workload}: creating simulation", file=sys.stderr, flush=True)
    sim = Sim(**cfg, sigma_mode=SIGMA_PER_CELL)
    t0 = time.perf_counter()
    sim.init_ic()
    torch.cuda.synchronize()
    print(f"[bench] initial conditions in {time.perf_counter() - t0:.2f} s, {sim.device_bytes / 1e9:.1f} GB on device",
          file=sys.stderr, flush=True)
    if args.warmup:
        sim.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] {args.warmup} warmup steps done", file=sys.stderr, flush=True)

    sim.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = dict(zip(KERNELS, (float(t) for t in sim.get_timings())))
    sim.set_profiling(False)
    print(f"[bench] {args.steps} timed steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    n = cfg["np_side"] ** 3
    value = n * args.steps / elapsed
    ab = algorithmic_bytes(cfg)
    dom = max(KERNELS, key=lambda k: ms[k])
    achieved = ab[dom] / (ms[dom] * 1e-3) / 1e9
    step_bytes = sum(ab.values())
    step_ms = sum(ms.values())
    k_step = elapsed / args.steps

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, args.cpu_sample_side, args.cpu_sample_steps)

    out = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": k_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {cfg['np_side']}^3 particles, {cfg['nm_side']}^3 FP32 mesh, "
                        f"{cfg['nc_side']}^3 coarse cells, x{cfg['x_bytes']}v{cfg['v_bytes']} codes, "
                        f"{cfg['box']:g} Mpc/h, Omega_m={cfg['omega_m']}, seeded BBKS Zel'dovich ICs at "
                        f"a={cfg['a_init']}, {cfg['n_steps']}-step schedule",
            "particles": n,
            "mesh": cfg["nm_side"],
            "coarse": cfg["nc_side"],
            "x_bytes": cfg["x_bytes"],
            "v_bytes": cfg["v_bytes"],
            "sigma": "per-cell",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": ab[dom],
            "avg_launch_ms": ms[dom],
        },
        "step_roofline": {
            "algorithmic_bytes": step_bytes,
            "achieved_GBs": step_bytes / k_step / 1e9,
            "frac": step_bytes / k_step / 1e9 / HBM_PEAK_GBS,
        },
        "kernels_ms": ms,
        "kernels_sum_ms": step_ms,
        "cpu_baseline": cpu,
    }
    sim.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
