#!/usr/bin/env python3
"""Benchmark: MLUPS of the TO-LES hot path on one MI355X.

Default workload: the D3Q19 turbulent-channel TO-LES, 96x48x48 fluid nodes
(x streamwise periodic, y halfway bounce-back walls, z periodic), FP32 shifted
populations with FP64 reductions, Smagorinsky substrate Cs = 0.1, 12 QoIs
({E, Z} x {B^2, B - B^2, I - B} + 6 mean-profile bands), h = 0 LRS closure
switched on at step 2500, 10000 steps.  Inputs are synthetic and seeded.

Prints one JSON line with the contract fields plus
  roofline:     the dominant kernel's achieved algorithmic bandwidth, timed
                live with HIP events on the stream it runs on;
  cpu_baseline: the FP64 CPU oracle timed on a bounded sample of the same
                workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def workload(name):
    import synth
    if name == "channel":
        nx, ny, nz = 96, 48, 48
        cfg, u0 = synth.channel_workload(nx, ny, nz, substrate=1, cmodel=0.1, seed=6)
        nb, dmin, dmax = synth.channel_bands(ny)
        C, mu, S = synth.lrs_model_channel(12, 7, 9)
        cargs = dict(mode="lrs", spinup=2500, C=C, mu=mu, Sigma=S, seed=8, nbands=nb, dmin=dmin, dmax=dmax)
        desc = ("D3Q19 channel TO-LES 96x48x48, FP32 shifted populations, Smagorinsky Cs=0.1, "
                "12 QoIs (E/Z x {B^2,B-B^2,I-B} + 6 mean-profile bands), LRS h=0 from step 2500")
        return dict(cfg=cfg, u0=u0, qois=synth.QOIS_3D, cargs=cargs, precision="fp32", desc=desc,
                    job_steps=10000, b_alg=232)
    if name == "channel_large":
        nx, ny, nz = 384, 192, 192
        cfg, u0 = synth.channel_workload(nx, ny, nz, substrate=1, cmodel=0.1, seed=6)
        nb, dmin, dmax = synth.channel_bands(ny)
        C, mu, S = synth.lrs_model_channel(12, 7, 9)
        cargs = dict(mode="lrs", spinup=250, C=C, mu=mu, Sigma=S, seed=8, nbands=nb, dmin=dmin, dmax=dmax)
        desc = ("D3Q19 channel TO-LES 384x192x192 (HBM-resident scale-up, same physics per cell), FP32 "
                "shifted populations, Smagorinsky Cs=0.1, 12 QoIs, LRS h=0 from step 250")
        return dict(cfg=cfg, u0=u0, qois=synth.QOIS_3D, cargs=cargs, precision="fp32", desc=desc,
                    job_steps=1000, b_alg=232)
    if name == "kolmogorov":
        n = 256
        cfg, _ = synth.kolmogorov_workload(n, tau=0.51, seed=2)
        u0 = synth.noise_velocity(2, (1, n, n), 1e-4, 2)
        C, mu, S = synth.lrs_model(2, 3, 4, 5)
        cargs = dict(mode="lrs", spinup=5000, C=C, mu=mu, Sigma=S, seed=12)
        desc = "D2Q9 Kolmogorov TO-LES 256x256, FP32 shifted, tau=0.51, E_B/Z_B QoIs, LRS h=0 from step 5000"
        return dict(cfg=cfg, u0=u0, qois=synth.QOIS_2D, cargs=cargs, precision="fp32", desc=desc,
                    job_steps=20000, b_alg=128)
    if name == "fine":
        nx, ny, nz = 480, 240, 240
        cfg, u0 = synth.channel_workload(nx, ny, nz, substrate=0, cmodel=0.0, seed=13)
        desc = "D3Q19 channel plain BGK 480x240x240, FP32 shifted populations"
        return dict(cfg=cfg, u0=u0, qois=None, cargs=None, precision="fp32", desc=desc,
                    job_steps=200, b_alg=152)
    raise SystemExit(f"unknown workload {name}")


def phase_bytes(w, ms, launches):
    """Algorithmic bytes per launch of each kernel phase (one read and one
    write of every field the phase needs, per cell)."""
    cfg = w["cfg"]
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    d = 2 if cfg["lattice"] == 0 else 3
    nc = 1 if d == 2 else 3
    Q = 9 if d == 2 else 19
    e = 8 if w["precision"] == "fp64" else 4
    to = w["qois"] is not None
    jv = jw = 0
    if to:
        deg = {"I": 0, "B": 1, "B2": 2, "BMID": 2, "IMB": 1}
        jv = max([2 * deg[f] for k, f, _ in w["qois"] if k == "E"] + [0])
        jw = max([2 * deg[f] for k, f, _ in w["qois"] if k == "Z"] + [0])
    per_cell = {
        "stream_collide": e * (2 * Q + ((1 + 2 * d) + (1 + d) if to else 0)),
        "curl": e * (d + nc),
        "binomial": e * 2 * (d + nc),
        "reduce": e * (d + jv * d + (jw + 1) * nc),
        "apply": e * (d + jv * d + (jw + 1) * nc + d),
        "solve": 0,
    }
    return {k: per_cell[k] * N for k in per_cell}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's job length)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="channel", choices=["channel", "channel_large", "kolmogorov", "fine"])
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path of this build is a single-GPU kernel set "
              "(an ensemble shards by member across GPUs without communication); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_32892_amd import lbm

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.empty(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: 5 x {args.copy_probe} MiB device-to-device copies", file=sys.stderr, flush=True)
        del a, b
    w = workload(args.workload)
    K = args.steps if args.steps is not None else w["job_steps"]
    W = args.warmup
    cfg = w["cfg"]
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]

    def make_run():
        spec = lbm.ClosureSpec(w["qois"], **w["cargs"]) if w["qois"] is not None else None
        r = lbm.Run(lbm.make_config(precision=w["precision"], **cfg), spec)
        r.init_velocity(w["u0"])
        return r

    run = make_run()
    run.step(W)
    run.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.step(K)
    status = run.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    mlups = N * K / dt / 1e6
    print(f"[bench] {args.workload}: {K} steps in {dt:.3f} s -> {mlups:.1f} MLUPS (status {status})",
          file=sys.stderr, flush=True)

    # live per-kernel timing (HIP events on the run's stream)
    prof = make_run()
    prof.step(W)
    ms, nl = prof.profile_phases(args.profile_steps)
    bytes_per_launch = phase_bytes(w, ms, nl)
    dom = max((k for k in ms if nl[k] > 0), key=lambda k: ms[k])
    dur_ms = ms[dom] / nl[dom]
    achieved = bytes_per_launch[dom] / (dur_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(dur_ms * 1e3, 2), "bytes_per_launch": bytes_per_launch[dom]}
    phases = {k: {"ms_per_step": round(ms[k], 5), "launches": nl[k]} for k in ms}

    out = {
        "metric": "MLUPS (D3Q19 TO-LES)" if args.workload == "channel" else f"MLUPS ({args.workload})",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(dt / K * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if w["precision"] != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "grid": [cfg["nx"], cfg["ny"], cfg["nz"]], "cells": N,
                   "job_steps": w["job_steps"], "parallelism": "single-gpu"},
        "hbm_fraction_step": {"b_alg_bytes_per_lup": w["b_alg"],
                              "frac": round(mlups * 1e6 * w["b_alg"] / (HBM_PEAK_GBS * 1e9), 4)},
        "roofline": roofline,
        "phases": phases,
    }

    if not args.no_cpu_baseline:
        import oracle
        import synth  # noqa: F401
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        o = oracle.Oracle(**cfg)
        o.init(w["u0"])
        if w["qois"] is not None:
            o.set_closure(oracle.make_closure(w["qois"], **w["cargs"]))
        t = time.perf_counter()
        o.step(1)
        one = time.perf_counter() - t
        n = max(1, min(2000, int(args.cpu_seconds / max(one, 1e-6))))
        t = time.perf_counter()
        o.step(n)
        tc = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(N * n / tc / 1e6, 4), "unit": "MLUPS", "cores": cores,
                               "kind": "oracle",
                               "sample": f"steps 1..{n} of the same workload (same grid, closure, inputs), "
                                         f"{tc:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
