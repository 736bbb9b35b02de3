#!/usr/bin/env python3
"""Splotch frame throughput on one MI355X (gfx950).

Workload: 10M particles in a Soneira-Peebles hierarchy (4 levels, 8
sub-clusters per level), two species with their own palettes, smoothing
length h = 1.3 n^(-1/3) from the local density (projected kernel radii from
sub-pixel to ~300 px over the poses), 1024 x 1024 images, 8 random camera
poses (some inside the cube), additive absorption-equals-emission transfer,
FP32 attributes.  One step renders all 8 poses; particles/s counts every input
particle of every pose.  Inputs are resident in device memory before timing.

Prints one JSON line.  `roofline` is for the dominant kernel, from HIP events
recorded inside the library around each stage during the timed steps;
`cpu_baseline` times the FP64 oracle on a bounded random subsample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "particles/s + HBM GB/s per frame; p50/p99 latency on mixed-view stream"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(n, seed=1001, pose_seed=2001, width=1024, height=1024, n_poses=8):
    from paper_1606_04427_amd import synth

    ps = synth.soneira_peebles(n, seed=seed)
    poses = synth.random_poses(n_poses, seed=pose_seed, width=width, height=height)
    looks, pals = [], []
    for k in range(2):
        s = ps.scalar[ps.species == k]
        looks.append(dict(log10=1, brightness=0.02 * (1 + k), lo=float(np.log10(s.min())),
                          hi=float(np.log10(s.max()))))
        pals.append(synth.palette(k))
    return ps, poses, looks, pals


def cpu_baseline(ps, poses, looks, pals, sample):
    from oracle import splref as R

    R.build(force=False)
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.sort(rng.choice(ps.n, sample, replace=False))
    sub = ps.subset(idx)
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    prm = R.params(R.ADD_AEQE, L)
    P = R.Particles(sub)
    t0 = time.perf_counter()
    for pose in poses:
        R.render(P, pose, prm)
    dt = time.perf_counter() - t0
    return {"value": sample * len(poses) / dt, "unit": "particles/s", "cores": 1,
            "kind": "oracle",
            "sample": f"random {sample}-particle subsample of the same set, all {len(poses)} poses, "
                      f"FP64 single-threaded C oracle, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build renders on exactly one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1606_04427_amd import binding as B

    t = time.time()
    ps, poses, looks, pals = workload(args.n)
    log(f"generated {ps.n} particles in {time.time() - t:.1f} s")
    dev = "cuda:0"
    ctx = B.Context(0)
    parts = B.DeviceParticles(ps, dev, "f32")
    prm = B.make_params(B.SPL_ADD_AEQE, B.Palettes(pals, dev), looks)
    imgs = [torch.empty((p.height, p.width, 3), dtype=torch.float32, device=dev) for p in poses]
    torch.cuda.synchronize()

    tile, cut = 16, 32.0
    if not args.no_autotune:
        tile, cut = ctx.spl_autotune(parts, poses[0], prm)
        log(f"autotune: tile {tile}, large cut {cut}")

    def step():
        for k, pose in enumerate(poses):
            ctx.spl_render(parts, pose, prm, out=imgs[k], stats=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = [ctx.spl_render(parts, p, prm, out=imgs[k])[1] for k, p in enumerate(poses)]
    ctx.spl_set_timing(True)
    ctx.spl_get_timing()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, by, frames = ctx.spl_get_timing()
    ctx.spl_set_timing(False)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps * len(poses) * ps.n / elapsed
    log(f"{args.steps} steps in {elapsed:.3f} s, {ms_per_step:.2f} ms/step, {value:.3e} particles/s")

    stages = {}
    for k, name in enumerate(B.STAGES):
        if frames:
            stages[name] = {"ms_per_frame": ms[k] / frames,
                            "GBps": (by[k] / (ms[k] * 1e-3) / 1e9) if ms[k] > 0 else None}
    kern = [k for k in range(len(B.STAGES)) if B.STAGES[k] not in ("host_gap_items",)]
    dom = max(kern, key=lambda k: ms[k])
    achieved = by[dom] / (ms[dom] * 1e-3) / 1e9 if ms[dom] > 0 else 0.0
    frame_bytes = sum(by[k] for k in kern) / max(frames, 1)
    dom_kernel = {"splat": "k_splat_add", "project": "k_project", "large_splat": "k_splat_large",
                  "scatter": "k_scatter", "count": "k_count", "finalise": "k_finalise",
                  "sort": "k_sort_chunks/k_merge_pass", "scan": "k_scan"}[B.STAGES[dom]]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom_kernel,
                "ms_per_launch": ms[dom] / max(frames, 1),
                "bytes_per_launch": by[dom] / max(frames, 1)}
    out = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Soneira-Peebles clustered set (4 levels x 8), 2 species, "
                               "1024x1024, 8 random poses, additive absorption=emission, FP32",
                   "n_particles": ps.n, "image": [1024, 1024], "poses": len(poses),
                   "tile": tile, "large_cut_px": cut},
        "hbm_GBps_per_frame": frame_bytes / (ms_per_step * 1e-3 / len(poses)) / 1e9,
        "ms_per_frame": ms_per_step / len(poses),
        "roofline": roofline,
        "stages": stages,
        "frames": [{"n_active": s["n_active"], "n_pairs": s["n_pairs"], "n_large": s["n_large"],
                    "n_large_pairs": s["n_large_pairs"]} for s in stats],
    }
    ctx.close()
    if not args.no_cpu_baseline:
        t = time.time()
        out["cpu_baseline"] = cpu_baseline(ps, poses, looks, pals, args.cpu_sample)
        log(f"cpu baseline in {time.time() - t:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
