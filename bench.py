#!/usr/bin/env python3
"""Throughput of the compressed particle-mesh step (1-byte positions and velocities) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3_pm2048]

One step = the whole hot path on the resident compressed state: integer CIC deposit, five-pass
FFT Poisson solve, force interpolation + kick + drift + re-encode (count pass, per-cell link and
scan, scatter pass). Initial conditions are generated on the GPU before the timed region. After W
warm-up steps (and the variant autotuner) the K steps right after them are timed as an early
window when the schedule leaves room, the run continues untimed, and the LAST K steps of the
schedule, ending at a = 1 where the particles are most clustered, are the timed region of `value`.
Prints one JSON line: particle-steps/s, the HBM roofline of the dominant kernel (algorithmic bytes
per launch over its HIP-event-timed duration, against the 8 TB/s peak; its vector-ALU view beside
it) and the oracle timed on the host cores on bounded samples of the workloads.
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
# 32-bit vector ALU operations per second without packed math: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz, an FMA counting as two (packed FP32, which would double it, is disabled in the compile flags)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# arithmetic operations per particle that the method itself needs in each move pass (decode,
# CIC weights, gradient interpolation, kick, drift, new cell, moments / encode)
ALGO_OPS_PER_PARTICLE = {"move_count": 136, "move_scatter": 147}
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


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (calibrated against a plain copy), or None when there is none or the kernel source has changed
    since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        for line in open(path):
            if not line.startswith("traffic-record:"):
                continue
            rec = dict(kv.split("=", 1) for kv in line.split()[1:])
            if rec.get("kernel") != kernel:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["sha256"]:
                return None
            kib = float(rec["fetch_kib"]) * float(rec["fetch_scale"]) + float(rec["write_kib"]) * float(rec["write_scale"])
            return kib * 1024.0
    return None


def measured_valu(kernel: str):
    """VALU instructions per launch of `kernel` from the committed rocprofv3 SQ counter summary, or
    None when there is none or the kernel source has changed since."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_instructions.md"))):
        for line in open(path):
            if not line.startswith("valu-record:"):
                continue
            rec = dict(kv.split("=", 1) for kv in line.split()[1:])
            if rec.get("kernel") != kernel:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["sha256"]:
                return None
            return float(rec["valu_insts"])
    return None


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(steps: dict):
    """The oracle (plain FP64 numpy PM on uncompressed particles, oracle.pm) timed on the host:
    the Poisson solve through scipy.fft with every host thread, CIC deposit and interpolation with
    numpy (one thread). Workloads: C1 (32^3 particles, 64^3 mesh), C2 (128^3, 256^3) and the 256^3
    sibling of the 2048^3 workload (same particle and mesh resolution), each from its own
    Zel'dovich initial conditions (untimed), `steps[name]` DKD steps timed after the initial half
    drift. `value` is the sibling's particle-steps/s: the rate at the headline workload's
    resolution."""
    from oracle import ic, pm
    from oracle.cosmology import Cosmology

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():  # the host's share of the machine, where it is set
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    pm.FFT_WORKERS = threads
    per = {}
    try:
        for name, k in steps.items():
            cfg = synth.WORKLOADS[name]
            cosmo = Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])
            x, p, _ = ic.zeldovich(cfg["np_side"], cfg["nm_side"], cfg["box"], cosmo, cfg["a_init"], cfg["seed"])
            run = pm.PMRun(x, p, cfg["nm_side"], cosmo, cfg["a_init"], cfg["a_final"], cfg["n_steps"],
                           cfg.get("spacing", 0))
            run.advance()  # initial half drift, untimed
            t0 = time.perf_counter()
            for _ in range(k):
                run.advance()
            dt = time.perf_counter() - t0
            n = cfg["np_side"] ** 3
            per[name] = {"steps": k, "seconds": dt, "ms_per_step": 1e3 * dt / k, "particle_steps_per_s": n * k / dt}
            print(f"[bench] oracle {name}: {k} steps in {dt:.1f} s", file=sys.stderr, flush=True)
    finally:
        pm.FFT_WORKERS = None
    sib = per["c3_sibling256"]
    return {
        "value": sib["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"FP64 numpy oracle (oracle.pm.PMRun, uncompressed particles): {sib['steps']} DKD steps of the "
                  f"256^3-particle, 256^3-mesh, 250 Mpc/h sibling of the 2048^3 workload (same particle and mesh "
                  f"resolution) in {sib['seconds']:.1f} s; scipy.fft with {threads} threads for the Poisson "
                  f"solve, numpy CIC deposit and interpolation on one thread",
        "cpu_model": host_cpu_model(),
        "host_cpus": threads,
        "workloads": per,
    }


def time_ensemble(cfgs, steps: int, warmup: int, label: str) -> dict:
    """cfgs stepped together with cube_batch_step (variants autotuned per box shape) in each launch
    mode -- kernels on per-box streams, one graph of per-box branches, one graph of ensemble
    launches (one launch per stage over all boxes) -- each mode continuing the run for `steps`
    steps, against the same boxes stepped one after another with cube_step over the steps the last
    mode ran; box 0's state after them is compared bit for bit."""
    import numpy as np
    import torch
    from paper_1712_06121_amd import Batch, Sim

    b = Batch(cfgs)
    b.init_ic()
    b.autotune()
    b.step(warmup)
    torch.cuda.synchronize()
    t_mode = {}
    modes = ((Batch.STREAMS, "streams"), (Batch.GRAPH, "graph"), (Batch.ENSEMBLE, "ensemble"))
    for mode, name in modes:
        b.set_mode(mode)
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        t_mode[name] = time.perf_counter() - t0
    ref0 = b.boxes[0].get_state()
    variants = sorted({(c["np_side"], tuple(box.variant.values())) for c, box in zip(cfgs, b.boxes)})
    dev_bytes = sum(box.device_bytes for box in b.boxes)
    b.close()
    print(f"[bench] {label} batch: {steps} steps in {t_mode}, variants {variants}", file=sys.stderr, flush=True)
    t_seq = 0.0
    same0 = None
    for i, c in enumerate(cfgs):
        with Sim(**c) as s:
            s.init_ic()
            s.step(warmup + (len(modes) - 1) * steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(steps)
            torch.cuda.synchronize()
            t_seq += time.perf_counter() - t0
            if i == 0:
                st = s.get_state()
                same0 = all(np.array_equal(st[k], ref0[k]) for k in ("cnt", "chi", "nu", "vc", "vs"))
    print(f"[bench] {label} sequential: {t_seq:.3f} s", file=sys.stderr, flush=True)
    best = min(t_mode, key=t_mode.get)
    return dict(t_mode=t_mode, t_seq=t_seq, best=best, same0=same0, variants=variants, dev_bytes=dev_bytes)


def bench_ensemble(args) -> dict:
    """The 64-box ensemble (synth.ensemble), timed in every batch launch mode against sequential
    cube_step (time_ensemble); beside it, 64 boxes of 32^3 particles (synth.ensemble_small), whose
    kernels alone leave most of the GPU idle."""
    cfgs = synth.ensemble(n_steps=50)
    total = sum(c["np_side"] ** 3 for c in cfgs)
    print(f"[bench] ensemble: {len(cfgs)} boxes, {total / 1e6:.1f} M particles", file=sys.stderr, flush=True)
    r = time_ensemble(cfgs, args.steps, args.warmup, "c4")
    small = synth.ensemble_small(n_steps=100)
    small_total = sum(c["np_side"] ** 3 for c in small)
    rs = time_ensemble(small, 4 * args.steps, args.warmup, "small")
    t_mode, t_seq, best_mode, same0, dev_bytes = r["t_mode"], r["t_seq"], r["best"], r["same0"], r["dev_bytes"]
    t_batch = t_mode[best_mode]
    step_bytes = sum(sum(algorithmic_bytes(c).values()) for c in cfgs)
    k_step = t_batch / args.steps
    return {
        "metric": "particle-steps/s",
        "value": total * args.steps / t_batch,
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
        "config": {"workload": f"c4_ensemble: {len(cfgs)} boxes of 64^3..256^3 particles (mesh 2x, coarse mesh/4), "
                               f"x1v1, n_s~U[0.9,1], sigma8~U[0.7,0.9], 50-step schedule; batched (fastest "
                               f"launch mode) vs sequential cube_step", "boxes": len(cfgs), "particles": total,
                   "device_bytes": dev_bytes},
        "roofline": {"bound": "hbm", "kernel": f"whole ensemble step ({best_mode})",
                     "achieved": step_bytes / k_step / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": step_bytes / k_step / 1e9 / HBM_PEAK_GBS, "traffic": None},
        "sequential": {"value": total * args.steps / t_seq, "seconds": t_seq},
        "speedup_vs_sequential": t_seq / t_batch,
        "speedup_vs_sequential_by_mode": {k: t_seq / v for k, v in t_mode.items()},
        "small_boxes": {"workload": f"{len(small)} boxes of 32^3 particles (mesh 64^3), x1v1",
                        "steps": 4 * args.steps, "particle_steps_per_s_by_mode":
                            {k: small_total * 4 * args.steps / v for k, v in rs["t_mode"].items()},
                        "sequential_particle_steps_per_s": small_total * 4 * args.steps / rs["t_seq"],
                        "speedup_vs_sequential_by_mode": {k: rs["t_seq"] / v for k, v in rs["t_mode"].items()},
                        "box0_bit_identical": rs["same0"]},
        "batch_seconds_by_mode": t_mode,
        "batch_mode": best_mode,
        "box0_bit_identical": same0,
        "cpu_baseline": None,
    }


def bench_serving(args) -> dict:
    """The serving stream (synth.serving_jobs): requests arrive in real time at their Poisson
    arrival times and are submitted to a cube_server; the loop polls it and records each job's
    completion. Latency = completion - arrival; throughput = all particle-steps / wall time from
    the first arrival to the last completion."""
    from paper_1712_06121_amd import Server

    jobs = synth.serving_jobs(n=args.serve_jobs)
    total_ps = sum(j["cfg"]["np_side"] ** 3 * j["cfg"]["n_steps"] for j in jobs)
    srv = Server(args.serve_budget_gb << 30, max_active=args.serve_slots, slice_steps=args.serve_slice)
    # warm-up: one job of each size (first launches load the kernels), untimed
    for i, side in enumerate((64, 128, 256)):
        cfg = dict(next(j["cfg"] for j in jobs if j["cfg"]["np_side"] == side), seed=1 + i)
        srv.submit(cfg, -1 - i)
    left = {-1, -2, -3}
    while left:
        for i in srv.poll():
            srv.release(i)
            left.discard(i)
        time.sleep(0.0005)
    print(f"[bench] serving {len(jobs)} jobs over {jobs[-1]['arrival']:.1f} s of arrivals", file=sys.stderr,
          flush=True)
    done = {}
    nxt = 0
    max_active = 0
    t0 = time.perf_counter()
    last_print = t0
    while len(done) < len(jobs):
        now = time.perf_counter() - t0
        while nxt < len(jobs) and jobs[nxt]["arrival"] <= now:
            srv.submit(jobs[nxt]["cfg"], nxt)
            nxt += 1
        fin = srv.poll()
        now = time.perf_counter() - t0
        for i in fin:
            st, rc = srv.status(i)
            if st != Server.FINISHED:
                raise RuntimeError(f"job {i} failed: {srv.job_error(i)}")
            done[i] = now
            srv.release(i)
        max_active = max(max_active, srv.stats()[1])
        if time.perf_counter() - last_print > 10.0:
            last_print = time.perf_counter()
            print(f"[bench] t={now:.1f} s: {len(done)} done, {nxt - len(done)} in the server", file=sys.stderr,
                  flush=True)
        if not fin:
            time.sleep(0.0002)
    srv.close()
    lat = sorted(done[i] - jobs[i]["arrival"] for i in range(len(jobs)))
    wall = max(done.values()) - jobs[0]["arrival"]
    p50, p99 = lat[len(lat) // 2], lat[min(len(lat) - 1, int(0.99 * len(lat)))]
    return {
        "metric": "particle-steps/s",
        "value": total_ps / wall,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": None,
        "warmup": None,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"c5_serving: {len(jobs)} Poisson arrivals at 20 jobs/s, 64^3/128^3/256^3 particles "
                               f"(p 0.5/0.35/0.15), mesh 2x, x1v1, sigma8~U[0.7,0.9], 50 steps",
                   "slots": args.serve_slots, "slice_steps": args.serve_slice,
                   "budget_GiB": args.serve_budget_gb},
        "latency_s": {"p50": p50, "p99": p99, "mean": sum(lat) / len(lat), "max": lat[-1]},
        "max_active_jobs": max_active,
        "offered_particle_steps_per_s": total_ps / jobs[-1]["arrival"],
        "roofline": None,
        "cpu_baseline": None,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3_pm2048",
                    choices=sorted(synth.WORKLOADS) + ["c4_ensemble", "c5_serving"])
    ap.add_argument("--serve-jobs", type=int, default=600, help="c5_serving: number of requests (2000 = 100 s)")
    ap.add_argument("--serve-slots", type=int, default=24)
    ap.add_argument("--serve-slice", type=int, default=5)
    ap.add_argument("--serve-budget-gb", type=int, default=160)
    ap.add_argument("--cpu-c1-steps", type=int, default=50, help="oracle steps timed on C1 (32^3 particles)")
    ap.add_argument("--cpu-c2-steps", type=int, default=4, help="oracle steps timed on C2 (128^3 particles)")
    ap.add_argument("--cpu-sibling-steps", type=int, default=2,
                    help="oracle steps timed on the 256^3 sibling of the 2048^3 workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-early-window", action="store_true", help="time only the last steps of the schedule")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel variants instead of timing the equivalent ones after warm-up")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain elementwise copy (torch.neg) over 1 GiB, the reference reading that "
                         "calibrates rocprofv3's FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (independent boxes "
              "would be placed whole on GPUs; one box would be cut into z-slabs). Use --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from paper_1712_06121_amd import SIGMA_PER_CELL, Sim

    torch.cuda.set_device(0)
    if args.workload == "c4_ensemble":
        print(json.dumps(bench_ensemble(args)))
        return 0
    if args.workload == "c5_serving":
        print(json.dumps(bench_serving(args)))
        return 0
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.neg(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: torch.neg over {src.numel() * 4} bytes read, {dst.numel() * 4} written",
              file=sys.stderr, flush=True)
        del src, dst
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
    if not args.no_autotune:
        t0 = time.perf_counter()
        sim.autotune()  # bit-identical variants; the fastest of each stage on this state
        torch.cuda.synchronize()
        print(f"[bench] autotune in {time.perf_counter() - t0:.1f} s: {sim.variant}", file=sys.stderr, flush=True)
        print(f"[bench] autotune times: {sim.autotune_report}", file=sys.stderr, flush=True)

    def timed_window(k):
        """k steps with per-kernel HIP events; (wall seconds, kernel ms per step, scale factors)."""
        a0 = sim.a
        sim.set_profiling(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(k)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ms_k = dict(zip(KERNELS, (float(x) for x in sim.get_timings())))
        sim.set_profiling(False)
        return el, ms_k, (a0, sim.a)

    # early window: the steps right after the warm-up (near-linear regime), when it does not overlap
    # the late window; then untimed steps up to the late window: the last `steps` steps of the
    # schedule, ending at a = 1 (the clustered regime), which give `value`
    early = None
    n_total = cfg["n_steps"]
    if args.warmup + 2 * args.steps <= n_total and not args.no_early_window:
        el, ms_e, a_e = timed_window(args.steps)
        early = {"steps": args.steps, "a": a_e, "ms_per_step": 1e3 * el / args.steps, "variants": dict(sim.variant),
                 "value": cfg["np_side"] ** 3 * args.steps / el, "kernels_ms": ms_e}
        print(f"[bench] early window a={a_e[0]:.3f}..{a_e[1]:.3f}: {1e3 * el / args.steps:.1f} ms/step",
              file=sys.stderr, flush=True)
    skip = n_total - args.steps - sim.steps_done
    while skip > 0:
        k = min(skip, 10)
        sim.step(k)
        torch.cuda.synchronize()
        skip -= k
        print(f"[bench] untimed steps to {sim.steps_done} (a={sim.a:.3f})", file=sys.stderr, flush=True)
    variants_early = sim.variant
    if not args.no_autotune:
        # the particles are far more clustered now: the variants are timed again on this state
        t0 = time.perf_counter()
        sim.autotune()
        torch.cuda.synchronize()
        print(f"[bench] autotune before the late window in {time.perf_counter() - t0:.1f} s: {sim.variant}",
              file=sys.stderr, flush=True)
        print(f"[bench] autotune times: {sim.autotune_report}", file=sys.stderr, flush=True)
    elapsed, ms, a_late = timed_window(args.steps)
    print(f"[bench] late window a={a_late[0]:.3f}..{a_late[1]:.3f}: {args.steps} timed steps in {elapsed:.3f} s",
          file=sys.stderr, flush=True)

    n = cfg["np_side"] ** 3
    value = n * args.steps / elapsed
    ab = algorithmic_bytes(cfg)
    dom = max(KERNELS, key=lambda k: ms[k])
    achieved = ab[dom] / (ms[dom] * 1e-3) / 1e9
    full = args.workload == "c3_pm2048"
    roofline = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": measured_traffic(dom) if full else None,
        "algorithmic_bytes_per_launch": ab[dom],
        "avg_launch_ms": ms[dom],
    }
    roofline_alu = None
    if dom in ALGO_OPS_PER_PARTICLE:
        # the move passes issue vector instructions back to back: their other bound is the vector ALU
        ops = ALGO_OPS_PER_PARTICLE[dom] * cfg["np_side"] ** 3
        tops = ops / (ms[dom] * 1e-3) / 1e12
        valu = measured_valu(dom) if full else None
        roofline_alu = {
            "bound": "alu",
            "kernel": dom,
            "achieved": tops,
            "peak": ALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": tops / ALU_PEAK_TOPS,
            "algorithmic_ops_per_launch": ops,
            "avg_launch_ms": ms[dom],
            "valu_instructions_per_launch": valu,
            "cycles_per_valu_issue_per_simd": (ms[dom] * 1e-3 * 2.4e9 / (valu / 1024)) if valu else None,
        }
    step_bytes = sum(ab.values())
    step_ms = sum(ms.values())
    k_step = elapsed / args.steps

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline({"c1_pm32": args.cpu_c1_steps, "c2_pm128": args.cpu_c2_steps,
                            "c3_sibling256": args.cpu_sibling_steps})

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
            "variants": sim.variant,
            "variants_early": variants_early,
            "device_bytes": sim.device_bytes,
        },
        "window": {"steps": args.steps, "a": a_late, "position": "last steps of the schedule, ending at a_final"},
        "early_window": early,
        "roofline": roofline,
        "roofline_alu": roofline_alu,
        "step_roofline": {
            "algorithmic_bytes": step_bytes,
            "achieved_GBs": step_bytes / k_step / 1e9,
            "frac": step_bytes / k_step / 1e9 / HBM_PEAK_GBS,
        },
        "kernels_ms": ms,
        "kernels_algorithmic_GBs": {k: ab[k] / (ms[k] * 1e-3) / 1e9 for k in KERNELS if ms[k] > 0},
        "kernels_sum_ms": step_ms,
        "cpu_baseline": cpu,
    }
    sim.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
