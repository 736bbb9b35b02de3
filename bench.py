#!/usr/bin/env python3
"""Splotch frame throughput on one MI355X (gfx950).

Default workload (additive): 10M particles in a Soneira-Peebles hierarchy (4
levels, 8 sub-clusters per level), two species with their own palettes,
smoothing length h = 1.3 n^(-1/3) from the local density (projected kernel
radii from sub-pixel to hundreds of px over the poses), 1024 x 1024 images, 8
random camera poses (some inside the cube), additive absorption-equals-emission
transfer, FP32 attributes.  One step renders all 8 poses with one call of the
batched entry point (one list-size synchronisation and one persistent splat
launch for the 8 views); the one-view-per-call path is timed beside it.
particles/s counts every input particle of every pose.  Inputs are resident in
device memory before timing.

Other workloads (--workload): `blobs` (100k particles in Gaussian blobs at
256^2, the small case, with the oracle timed on the same frame), `sorted` (the
same 10M set with absorption,
depth-sorted transfer, one 2048 x 2048 view), `batched` (200M particles with
BF16 or FP16 attributes, 64 views of 4096^2 and 1024^2 in batched launches),
`serving` (100M resident particles, a Poisson stream of mixed-size views).

Prints one JSON line.  `roofline` is for the dominant kernel, from HIP events
recorded inside the library around each stage during the timed steps;
`cpu_baseline` times the FP64 oracle on a bounded random subsample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Operations per Gaussian pixel update (additive modes): about 11 FP32
# operations (the offsets of the pixel centre from the particle, the squared
# distance, the truncation test, three colour multiply-adds counted as two
# operations each) plus one exponential, counted as one operation
FLOPS_PER_UPDATE = 12.0
# Operations per pixel update of the depth-sorted composite: the additive
# count of 11, the optical depth a w (1), the degree-5 polynomial for
# phi(x) = (1 - exp(-x)) / x (five multiply-adds, 10), exp(-x) - 1 from it
# (1), the weight T w phi (2) and the transmittance update (one
# multiply-add, 2), plus the Gaussian's exponential (1).  Optical depths of
# 1/2 and more take an exponential and a reciprocal instead of the polynomial.
FLOPS_PER_COMPOSITE_UPDATE = 28.0
METRIC = "particles/s + HBM GB/s per frame; p50/p99 latency on mixed-view stream"
KERNEL_OF_STAGE = {"splat": "k_splat_add", "project": "k_project", "large_splat": "k_splat_large",
                   "scatter": "k_scatter", "count": "k_count", "finalise": "k_finalise",
                   "sort": "k_sort_chunks/k_merge_pass", "scan": "k_scan"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def looks_for(ps, scale=1.0, palette_offset=0):
    from paper_1606_04427_amd import synth

    looks, pals = [], []
    for k in range(2):
        s = ps.scalar[ps.species == k]
        looks.append(dict(log10=1, brightness=0.02 * (1 + k) * scale, lo=float(np.log10(s.min())),
                          hi=float(np.log10(s.max()))))
        pals.append(synth.palette((k + palette_offset) % 2))
    return looks, pals


def workload(n, seed=1001, pose_seed=2001, width=1024, height=1024, n_poses=8, absorption=False):
    from paper_1606_04427_amd import synth

    ps = synth.soneira_peebles(n, seed=seed, absorption=absorption)
    poses = synth.random_poses(n_poses, seed=pose_seed, width=width, height=height)
    looks, pals = looks_for(ps)
    return ps, poses, looks, pals


def cpu_baseline(ps, poses, looks, pals, sample, mode):
    from oracle import splref as R

    R.build(force=False)
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.sort(rng.choice(ps.n, sample, replace=False))
    sub = ps.subset(idx)
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    prm = R.params(mode, L)
    P = R.Particles(sub)
    t0 = time.perf_counter()
    for pose in poses:
        R.render(P, pose, prm)
    dt = time.perf_counter() - t0
    return {"value": sample * len(poses) / dt, "unit": "particles/s", "cores": 1,
            "kind": "oracle",
            "sample": f"random {sample}-particle subsample of the same set, {len(poses)} pose(s), "
                      f"FP64 single-threaded C oracle, {dt:.1f} s"}


def cpu_baseline_all_cores(ps, poses, looks, pals, sample, mode):
    """The same oracle runs on several host threads, one pose each (the C
    oracle releases the interpreter lock and keeps no global state)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import splref as R

    R.build(force=False)
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.sort(rng.choice(ps.n, sample, replace=False))
    sub = ps.subset(idx)
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    prm = R.params(mode, L)
    P = R.Particles(sub)
    threads = max(1, min(len(poses), os.cpu_count() or 1, 16))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda pose: R.render(P, pose, prm), poses))
    dt = time.perf_counter() - t0
    return {"value": sample * len(poses) / dt, "unit": "particles/s", "cores": threads,
            "kind": "oracle",
            "sample": f"random {sample}-particle subsample, {len(poses)} pose(s) on {threads} host "
                      f"threads, {dt:.1f} s"}


def box_pixels(rec, width, height, cut):
    """Pixels inside the clipped integer box of every small particle (R <= cut
    or no cut): the Gaussian updates an exact splat must evaluate."""
    r = rec.reshape(-1, 8).astype(np.float64)
    sig = r[:, 4]
    R = 3.0 * sig
    X = r[:, 0] + r[:, 1]
    Y = r[:, 2] + r[:, 3]
    small = sig > 0
    if cut > 0:
        small &= R <= cut
    # clip each end on its own side only, so that a box wholly off the image
    # stays empty
    i0 = np.maximum(np.ceil(X - R - 0.5), 0)
    i1 = np.minimum(np.floor(X + R - 0.5), width - 1)
    j0 = np.maximum(np.ceil(Y - R - 0.5), 0)
    j1 = np.minimum(np.floor(Y + R - 0.5), height - 1)
    area = np.maximum(i1 - i0 + 1, 0) * np.maximum(j1 - j0 + 1, 0)
    return float(area[small].sum()), int(small.sum())


def radius_range(rec, k_sigma=1.0 / 3.0, sigma_min=0.5):
    """Realised projected radius rho (px) over the active records of a view:
    sigma = sqrt((k_sigma rho)^2 + sigma_min^2) inverted for rho."""
    sig = np.asarray(rec, np.float64).reshape(-1, 8)[:, 4]
    sig = sig[sig > 0]
    if sig.size == 0:
        return None
    rho = np.sqrt(np.maximum(sig * sig - sigma_min * sigma_min, 0.0)) / k_sigma
    q = np.percentile(rho, [50, 99])
    return {"min": float(rho.min()), "p50": float(q[0]), "p99": float(q[1]),
            "max": float(rho.max())}


def footprint(box_px, small):
    """Box pixels per small particle over several views: both lists hold one
    entry per view, so the ratio of their sums is the mean over every
    (particle, view) pair."""
    return float(sum(box_px)) / max(int(sum(small)), 1)


def timed_steps(ctx, step, steps, warmup, torch):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.spl_set_timing(True)
    ctx.spl_get_timing()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, by, frames = ctx.spl_get_timing()
    ctx.spl_set_timing(False)
    return elapsed, ms, by, frames


def stage_table(B, ms, by, frames):
    out = {}
    for k, name in enumerate(B.STAGES):
        if frames:
            out[name] = {"ms_per_frame": ms[k] / frames,
                         "GBps": (by[k] / (ms[k] * 1e-3) / 1e9) if ms[k] > 0 else None}
    return out


def roofline_for(B, ms, by, launches, updates_per_launch=None, flops_per_update=FLOPS_PER_UPDATE):
    """Roofline of the dominant stage; `launches` is the number of launches
    the accumulated stage times cover (frames for one view per call, steps
    for the batched call)."""
    kern = [k for k in range(len(B.STAGES)) if B.STAGES[k] not in ("host_gap_items",)]
    dom = max(kern, key=lambda k: ms[k])
    name = B.STAGES[dom]
    frames = launches
    per_launch = ms[dom] / max(frames, 1)
    updates_per_frame = updates_per_launch
    if name == "splat" and updates_per_frame:
        # the splat evaluates a Gaussian per pixel of each particle's box: its
        # bound is the vector ALU, not HBM
        achieved = flops_per_update * updates_per_frame / (per_launch * 1e-3) / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                "kernel": KERNEL_OF_STAGE[name], "ms_per_launch": per_launch,
                "updates_per_launch": updates_per_frame,
                "flops_per_update": flops_per_update,
                "hbm_GBps": by[dom] / (ms[dom] * 1e-3) / 1e9,
                "hbm_frac": by[dom] / (ms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "bytes_per_launch": by[dom] / max(frames, 1)}
    achieved = by[dom] / (ms[dom] * 1e-3) / 1e9 if ms[dom] > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": KERNEL_OF_STAGE[name],
            "ms_per_launch": per_launch, "bytes_per_launch": by[dom] / max(frames, 1)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_splat_additive_10M_1024x1024.txt")


def source_digest(names):
    import hashlib

    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1606_04427_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, n, tile, cut):
    """HBM bytes per launch of the dominant kernel from the committed counter
    profile (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when
    there is none for this kernel, workload and configuration, or when the
    kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.loads(f.read().split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    if (rec.get("kernel") != kernel or rec.get("n") != n or rec.get("tile") != tile
            or rec.get("cut") != cut or rec.get("digest") != source_digest(rec["sources"])):
        return None
    return rec["bytes_per_launch"]


def base_record(args, value, ms_per_step, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


# ----------------------------------------------------------------------------
def run_additive(args, torch, B):
    t = time.time()
    ps, poses, looks, pals = workload(args.n or 10_000_000)
    log(f"generated {ps.n} particles in {time.time() - t:.1f} s")
    dev = "cuda:0"
    ctx = B.Context(0)
    parts = B.Dataset(ctx, ps, "f32")
    pal_d = B.Palettes(pals, dev)
    prm = B.make_params(B.SPL_ADD_AEQE, pal_d, looks)
    imgs = [torch.empty((p.height, p.width, 3), dtype=torch.float32, device=dev) for p in poses]
    torch.cuda.synchronize()

    tuned = None
    if args.tile:
        # fixed configuration (profiling runs repeat the tuned one)
        prm = B.make_params(B.SPL_ADD_AEQE, pal_d, looks, tile=args.tile, large_cut=args.cut)
    elif not args.no_autotune:
        # the tile size and large-particle cut are tuned per pose: the radii a
        # pose projects decide whether the large-particle path pays
        tuned = [ctx.spl_autotune(parts, p, prm) for p in poses]
        log(f"autotune per pose (tile, cut): {tuned}")

    prms = [prm] * len(poses)

    # one step: all poses in one call of the batched entry point (one list-size
    # synchronisation, one persistent splat launch per tile size)
    def step():
        ctx.spl_render_batch_dataset(parts, poses, prms, outs=imgs, stats=False)

    elapsed, ms, by, frames = timed_steps(ctx, step, args.steps, args.warmup, torch)
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps * len(poses) * ps.n / elapsed
    log(f"{args.steps} steps in {elapsed:.3f} s, {ms_per_step:.2f} ms/step, {value:.3e} particles/s")
    _, bstats = ctx.spl_render_batch_dataset(parts, poses, prms, outs=imgs)
    tiles_used = sorted({s["tile"] for s in bstats})

    # outside the timed region: per-pose statistics and the Gaussian updates
    # the splat had to evaluate (from the device's own records)
    stats = [ctx.spl_render_dataset(parts, p, prm, out=imgs[k])[1] for k, p in enumerate(poses)]
    pose_updates, pose_small, pose_rho = [], [], []
    for k, p in enumerate(poses):
        rec, _ = ctx.spl_project(parts, p, prm)
        rh = rec.cpu().numpy()
        u, s = box_pixels(rh, p.width, p.height, stats[k]["large_cut"])
        pose_updates.append(u)
        pose_small.append(s)
        pose_rho.append(radius_range(rh))
        del rec, rh
    updates = float(sum(pose_updates))
    # one persistent splat launch per step covers all poses (when they share a
    # tile size)
    roofline = roofline_for(B, ms, by, args.steps * len(tiles_used), updates / len(tiles_used))
    roofline["kernel"] = "k_splat_add_views" if roofline["kernel"] == "k_splat_add" else roofline["kernel"]
    roofline["traffic"] = measured_traffic(roofline["kernel"], ps.n, bstats[0]["tile"],
                                           bstats[0]["large_cut"])

    # the same step one view per call, with the library's per-stage events
    def pstep():
        for k, pose in enumerate(poses):
            ctx.spl_render_dataset(parts, pose, prm, out=imgs[k], stats=False)

    p_elapsed, p_ms, p_by, p_frames = timed_steps(ctx, pstep, args.steps, args.warmup, torch)
    per_view = {"ms_per_step": 1e3 * p_elapsed / args.steps,
                "particles_per_s": args.steps * len(poses) * ps.n / p_elapsed,
                "stages": stage_table(B, p_ms, p_by, p_frames)}
    log(f"one view per call: {per_view['ms_per_step']:.2f} ms/step")
    # per pose: splat time and the footprint that drives it, and the frame
    # time at each large-particle cut (the evidence behind the tuned choice)
    si, li = B.STAGES.index("splat"), B.STAGES.index("large_splat")
    per_pose = []
    for k, p in enumerate(poses):
        def timed(q, reps=3):
            ctx.spl_render_dataset(parts, p, q, out=imgs[k], stats=False)
            ctx.spl_set_timing(True)
            ctx.spl_get_timing()
            for _ in range(reps):
                ctx.spl_render_dataset(parts, p, q, out=imgs[k], stats=False)
            pm, _, pf = ctx.spl_get_timing()
            ctx.spl_set_timing(False)
            return pm, max(pf, 1)

        pm, pf = timed(prm)
        row = {"n_active": stats[k]["n_active"], "n_pairs": stats[k]["n_pairs"],
               "n_large": stats[k]["n_large"], "tile": stats[k]["tile"],
               "large_cut": stats[k]["large_cut"], "rho_px": pose_rho[k],
               "box_px": pose_updates[k],
               "box_px_per_active": pose_updates[k] / max(stats[k]["n_active"], 1),
               "frame_ms": sum(pm) / pf, "splat_ms": pm[si] / pf}
        if not args.no_cut_table:
            cuts = {}
            for cut in (16.0, 32.0, 64.0, 128.0, -1.0):
                q = B.make_params(B.SPL_ADD_AEQE, pal_d, looks, tile=stats[k]["tile"],
                                  large_cut=cut)
                cm, cf = timed(q)
                cuts["off" if cut < 0 else f"{cut:g}"] = {
                    "frame_ms": sum(cm) / cf, "splat_ms": cm[si] / cf,
                    "large_splat_ms": cm[li] / cf}
            row["frame_ms_by_cut"] = cuts
        per_pose.append(row)
    log("per pose: " + json.dumps([{k: v for k, v in r.items() if k != "rho_px"}
                                    for r in per_pose])[:2000])

    # the batched step replayed as a captured graph
    graphs = None
    if not args.no_graph_replay:
        ctx.spl_set_option(B.SPL_OPT_GRAPHS, 1)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.spl_set_option(B.SPL_OPT_GRAPHS, 0)
        graphs = {"ms_per_step": 1e3 * dt / args.steps,
                  "particles_per_s": args.steps * len(poses) * ps.n / dt}
        log("graph replay: " + json.dumps(graphs))
    if args.copy_probe_gib:
        # a plain device copy of known size: the reference point that scales
        # the HBM byte counters of a profiling run
        nb = int(args.copy_probe_gib * (1 << 30)) // 4
        src = torch.ones(nb, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the additive image in list order (run-to-run bit-identical): the same
    # poses one view per call, against the unordered one-view-per-call step
    det_rec = None
    if not args.no_deterministic_leg:
        det_rec = deterministic_leg(args, torch, B, ctx, parts, poses, pal_d, looks, imgs,
                                    per_view["ms_per_step"])
        log("deterministic: " + json.dumps({k: v for k, v in det_rec.items() if k != "stages"}))

    # out-of-core rendering of the same set from page-locked host memory, in
    # chunks through two device buffers (copies overlapped with rendering)
    stream_rec = None
    if not args.no_stream:
        stream_rec = stream_leg(args, torch, B, ctx, ps, poses[0], prm, parts)
        log("out-of-core: " + json.dumps(stream_rec))

    # bandwidth probe: the same particle count with small radii (0.5-8 px,
    # the small blob case's distribution) at 1024 x 1024
    probe = None
    if not args.no_probe:
        probe = bandwidth_probe(args, torch, B, ctx, ps.n)
        log("bandwidth probe: " + json.dumps(probe))

    frame_bytes = sum(by[k] for k in range(len(B.STAGES)) if B.STAGES[k] != "host_gap_items")
    frame_bytes /= max(frames, 1)
    out = base_record(args, value, ms_per_step, "f32", {
        "workload": "Soneira-Peebles clustered set (4 levels x 8), 10M particles, 2 species, "
                    "1024x1024, 8 random poses per step in one batched call, additive "
                    "absorption=emission, FP32",
        "n_particles": ps.n, "image": [1024, 1024], "poses": len(poses),
        "tiles": tiles_used, "tuned_per_pose": tuned})
    out.update({
        "hbm_GBps_per_frame": frame_bytes / (ms_per_step * 1e-3 / len(poses)) / 1e9,
        "ms_per_frame": ms_per_step / len(poses),
        "roofline": roofline,
        "stages": stage_table(B, ms, by, frames),
        "one_view_per_call": per_view,
        "batched_graph_replay": graphs,
        "per_pose": per_pose,
        "out_of_core": stream_rec,
        "deterministic": det_rec,
        "bandwidth_probe": probe,
        "mean_box_px_per_small_particle": footprint(pose_updates, pose_small),
        "frames": [{"n_active": s["n_active"], "n_pairs": s["n_pairs"], "n_large": s["n_large"],
                    "n_large_pairs": s["n_large_pairs"], "tile": s["tile"],
                    "large_cut": s["large_cut"]} for s in bstats],
    })
    parts.close()
    if not args.no_sorted_leg:
        out["sorted"] = sorted_leg(args, torch, B, ctx)
        log("sorted: " + json.dumps({k: v for k, v in out["sorted"].items() if k != "stages"}))
    ctx.close()
    if not args.no_serving:
        out["serving"] = serving_leg(args, torch, B)
    if not args.no_batched_leg:
        t = time.time()
        out["batched_200M"] = batched_leg(args, torch, B)
        log(f"batched 200M leg in {time.time() - t:.1f} s")
    if not args.no_orbit_leg:
        t = time.time()
        out["orbit"] = orbit_leg(args, torch, B)
        log(f"orbit leg in {time.time() - t:.1f} s")
    if not args.no_cpu_baseline:
        t = time.time()
        out["cpu_baseline"] = cpu_baseline(ps, poses, looks, pals, args.cpu_sample or 5_000_000,
                                           B.SPL_ADD_AEQE)
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(
            ps, poses, looks, pals, args.cpu_sample or 5_000_000, B.SPL_ADD_AEQE)
        log(f"cpu baseline in {time.time() - t:.1f} s")
    return out


def deterministic_leg(args, torch, B, ctx, parts, poses, pal_d, looks, imgs, free_ms):
    """The additive frame with spl_params.deterministic = 1 (tile lists in
    ascending particle index, each list summed in that order): ms per step of
    the poses one view per call, its stage times, whether two renders of a
    pose agree bit for bit, and its difference from the unordered image."""
    prm = B.make_params(B.SPL_ADD_AEQE, pal_d, looks, deterministic=1)
    free = B.make_params(B.SPL_ADD_AEQE, pal_d, looks)

    def step():
        for k, pose in enumerate(poses):
            ctx.spl_render_dataset(parts, pose, prm, out=imgs[k], stats=False)

    elapsed, ms, by, frames = timed_steps(ctx, step, args.steps, args.warmup, torch)
    ms_per_step = 1e3 * elapsed / args.steps
    same, err = [], []
    for k in (0, len(poses) // 2):
        a = ctx.spl_render_dataset(parts, poses[k], prm)[0].cpu().numpy()
        ctx.spl_render_dataset(parts, poses[k], free, out=imgs[k], stats=False)
        u = imgs[k].cpu().numpy()
        b = ctx.spl_render_dataset(parts, poses[k], prm)[0].cpu().numpy()
        same.append(bool(np.array_equal(a.view(np.uint32), b.view(np.uint32))))
        den = float(np.linalg.norm(u.astype(np.float64)))
        err.append(float(np.linalg.norm(a.astype(np.float64) - u)) / max(den, 1e-300))
    return {"ms_per_step": ms_per_step,
            "particles_per_s": args.steps * len(poses) * parts.n / elapsed,
            "vs_unordered_one_view_per_call": free_ms / ms_per_step,
            "bit_identical_repeats": same, "rel_l2_vs_unordered": err,
            "stages": stage_table(B, ms, by, frames)}


def orbit_leg(args, torch, B):
    """The orbit animation in the default run: 55M particles, 100-frame orbit
    at 1024^2 per batched call (1 warm-up, 2 timed steps, the library's tile
    and cut), and the 6-pose far-to-near sweep one view per call."""
    import copy

    a = copy.copy(args)
    a.n, a.steps, a.warmup, a.no_autotune, a.no_cpu_baseline = 0, 2, 1, True, True
    out = run_orbit(a, torch, B)
    return {"workload": out["config"]["workload"], "particles_per_s": out["value"],
            "batch_workspace_gib": out["config"]["batch_workspace_gib"],
            "ms_per_frame": out["ms_per_frame"], "sweep": out["sweep"]}


def batched_leg(args, torch, B):
    """The batched reduced-precision configuration in the default run: 200M
    particles with BF16 attributes, 64 views alternating 4096^2 and 1024^2 in
    one call, the tile and cut per image size the batched workload's own
    tuning picks (16 px, no large path at 4096^2; 16 px, 64 px cut at
    1024^2), 2 timed steps; error against the FP64 oracle on two views of a
    1M-particle subsample."""
    import copy

    a = copy.copy(args)
    a.n, a.dtypes, a.steps, a.views, a.error_views = 0, "bf16", 2, 64, 2
    out = run_batched(a, torch, B, fixed={4096: (16, -1.0), 1024: (16, 64.0)})
    v = out["variants"]["bf16"]
    return {"workload": out["config"]["workload"], "dtype": "bf16",
            "batch_workspace_gib": out["config"]["batch_workspace_gib"],
            "particle_views_per_s": out["value"], "ms_per_step": out["ms_per_step"],
            "batched_graph": v["batched_graph"], "per_view_calls": v["per_view"],
            "stages_ms_per_step": v["stages_ms_per_step"],
            "error_vs_fp64_oracle_1M_subsample": v["error_vs_fp64_oracle_1M_subsample"],
            "tile_cut_by_size": v["tile_cut_by_size"]}


def sorted_leg(args, torch, B, ctx):
    """The depth-sorted transfer config: the same clustered set with
    absorption U[0.01, 0.5], one 2048 x 2048 view (the first pose), tuned
    tile; particles/s, stage times and the dominant kernel's roofline."""
    ps, poses, looks, pals = workload(args.n or 10_000_000, width=2048, height=2048,
                                      absorption=True)
    parts = B.Dataset(ctx, ps, "f32")
    prm = B.make_params(B.SPL_SORTED, B.Palettes(pals), looks)
    pose = poses[0]
    tile = None if args.no_autotune else ctx.spl_autotune(parts, pose, prm)[0]
    img = torch.empty((pose.height, pose.width, 3), dtype=torch.float32, device="cuda:0")

    def step():
        ctx.spl_render_dataset(parts, pose, prm, out=img, stats=False)

    elapsed, ms, by, frames = timed_steps(ctx, step, args.steps, args.warmup, torch)
    st = ctx.spl_render_dataset(parts, pose, prm, out=img)[1]
    # outside the timed region: the pixel updates the composite evaluates (every
    # listed particle's clipped box; sorted mode has no large-particle cut)
    rec, _ = ctx.spl_project(parts, pose, prm)
    updates, _ = box_pixels(rec.cpu().numpy(), pose.width, pose.height, 0.0)
    del rec
    roof = roofline_for(B, ms, by, frames, updates, FLOPS_PER_COMPOSITE_UPDATE)
    if roof["kernel"] == "k_splat_add":
        roof["kernel"] = "k_composite"  # the sorted mode's splat stage
    parts.close()
    return {"workload": f"{ps.n} clustered particles with absorption U[0.01,0.5], 2048x2048, "
                        "depth-sorted transfer, FP32",
            "particles_per_s": args.steps * ps.n / elapsed,
            "ms_per_frame": 1e3 * elapsed / args.steps, "tile": st["tile"],
            "n_active": st["n_active"], "n_pairs": st["n_pairs"], "roofline": roof,
            "stages": stage_table(B, ms, by, frames)}


def stream_leg(args, torch, B, ctx, ps, pose, prm, parts):
    """Out-of-core rendering: the set from page-locked host memory in chunks
    (Sect. 3.1's double-buffered copies).  Reports the streamed frame time,
    the copy time of the same bytes alone and the resident frame time, and the
    share of the copy time the overlap hides."""
    chunk = args.stream_chunk
    host = B.PinnedParticles(ps)
    img = torch.empty((pose.height, pose.width, 3), dtype=torch.float32, device="cuda:0")
    reps = max(3, args.steps // 2)

    def time_it(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    streamed = time_it(lambda: ctx.spl_render_stream(host, chunk, pose, prm, out=img, stats=False))
    resident = time_it(lambda: ctx.spl_render_dataset(parts, pose, prm, out=img, stats=False))
    # the same copies alone: per chunk, one host-to-device copy per array
    # (positions, smoothing length, intensity, scalar, species), pinned source
    nbytes = ps.n * (12 + 12 + 1)
    sizes = [4, 4, 4, 4, 4, 4, 1]
    srcs = [torch.empty(ps.n * b, dtype=torch.uint8).pin_memory() for b in sizes]
    dsts = [torch.empty(chunk * b, dtype=torch.uint8, device="cuda:0") for b in sizes]

    def copies():
        for k0 in range(0, ps.n, chunk):
            m = min(chunk, ps.n - k0)
            for b, src, dst in zip(sizes, srcs, dsts):
                dst[: m * b].copy_(src[k0 * b:(k0 + m) * b], non_blocking=True)

    copy = time_it(copies)
    del srcs, dsts
    ref = ctx.spl_render_stream(host, chunk, pose, prm, stats=False)[0].cpu().numpy()
    host.close()
    # the overlap saves copy + resident - streamed against copying, then
    # rendering; at most the render time can hide under the copies
    overlap = copy + resident - streamed
    # the same frame from BF16 attributes in host memory (rounded to nearest
    # even here, by the caller): 19 bytes per particle over the link instead
    # of 25; its error against the FP32 frame
    def bf16_bits(a):
        u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
        return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)

    hb = B.PinnedParticles(ps, {"h": bf16_bits(ps.h), "intensity": bf16_bits(ps.intensity),
                                "scalar": bf16_bits(ps.scalar)}, B.SPL_BF16)
    streamed_bf16 = time_it(lambda: ctx.spl_render_stream(hb, chunk, pose, prm, out=img,
                                                           stats=False))
    got = ctx.spl_render_stream(hb, chunk, pose, prm, stats=False)[0].cpu().numpy()
    hb.close()
    err = float(np.linalg.norm((got - ref).astype(np.float64)) /
                max(float(np.linalg.norm(ref.astype(np.float64))), 1e-300))
    return {"chunk_particles": chunk, "chunks": -(-ps.n // chunk), "bytes_copied": nbytes,
            "streamed_ms": streamed, "resident_ms": resident, "copies_alone_ms": copy,
            "copy_GBps": nbytes / (copy * 1e-3) / 1e9, "overlap_ms": overlap,
            "render_hidden_fraction": overlap / resident if resident > 0 else 0.0,
            "particles_per_s": ps.n / (streamed * 1e-3),
            "bf16": {"bytes_copied": ps.n * (12 + 6 + 1), "streamed_ms": streamed_bf16,
                     "particles_per_s": ps.n / (streamed_bf16 * 1e-3),
                     "rel_l2_vs_f32": err}}


def bandwidth_probe(args, torch, B, ctx, n):
    """n blob particles whose projected radii follow the small case's
    log-normal distribution (0.5-8 px) at 1024 x 1024: the regime where the
    splat moves the most bytes per Gaussian evaluation."""
    from paper_1606_04427_amd import synth

    pb = synth.blobs(n, seed=1000)
    # the blob recipe sizes h for a 256-px view; four times the pixels per
    # world unit at 1024 px, so h / 4 keeps the radii in px
    pb.h = (pb.h / 4.0).astype(np.float32)
    bparts = B.Dataset(ctx, pb, "f32")
    s_ = pb.scalar[pb.scalar > 0]
    blook = [dict(log10=1, brightness=0.3, lo=float(np.log10(s_.min())),
                  hi=float(np.log10(s_.max())))]
    bprm = B.make_params(B.SPL_ADD_AEQE, B.Palettes([synth.palette(0)]), blook, tile=16,
                         large_cut=-1.0)
    bcam = synth.blobs_camera(1024, 1024)
    bimg = torch.empty((1024, 1024, 3), dtype=torch.float32, device="cuda:0")
    for _ in range(2):
        ctx.spl_render_dataset(bparts, bcam, bprm, out=bimg, stats=False)
    ctx.spl_set_timing(True)
    ctx.spl_get_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.spl_render_dataset(bparts, bcam, bprm, out=bimg, stats=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pm, pby, pf = ctx.spl_get_timing()
    ctx.spl_set_timing(False)
    st = ctx.spl_render_dataset(bparts, bcam, bprm, out=bimg)[1]
    rec, _ = ctx.spl_project(bparts, bcam, bprm)
    upd, small = box_pixels(rec.cpu().numpy(), 1024, 1024, -1.0)
    del rec
    bparts.close()
    si = B.STAGES.index("splat")
    splat_s = pm[si] / pf * 1e-3
    return {"workload": f"{pb.n} particles in 64 Gaussian blobs, projected radii 0.5-8 px "
                        "(log-normal about 2 px), 1024x1024, fixed camera, additive",
            "particles_per_s": args.steps * pb.n / dt, "ms_per_frame": 1e3 * dt / args.steps,
            "n_pairs": st["n_pairs"], "box_px_per_particle": upd / max(small, 1),
            "splat_ms": pm[si] / pf, "splat_GBps": pby[si] / pf / splat_s / 1e9,
            "splat_hbm_frac": pby[si] / pf / splat_s / 1e9 / HBM_PEAK_GBS,
            "splat_TFLOPs": FLOPS_PER_UPDATE * upd / splat_s / 1e12,
            "stages_ms": {B.STAGES[i]: pm[i] / pf for i in range(len(B.STAGES))}}


# ----------------------------------------------------------------------------
def run_orbit(args, torch, B):
    """Animation workload of the paper's benchmark shape (Sect. 4.1, Sect. 4.3):
    a 55M-particle clustered set (about 10% of it the second species), a
    100-frame camera orbit at 1024x1024 rendered through the batched entry
    point, and a far-to-near sweep of 6 poses timed one view per call, with
    the time per particle against the mean projected radius."""
    from paper_1606_04427_amd import synth

    n = args.n or 55_000_000
    t = time.time()
    ps = synth.soneira_peebles(n, seed=1005)
    log(f"generated {ps.n} particles in {time.time() - t:.1f} s")
    orbit = synth.orbit_poses(100)
    sweep = synth.sweep_poses(6)
    looks, pals = looks_for(ps)
    dev = "cuda:0"
    ctx = B.Context(0)
    ctx.spl_set_option(B.SPL_OPT_BATCH_BYTES, args.batch_gib << 30)
    parts = B.DeviceParticles(ps, dev)
    prm = B.make_params(B.SPL_ADD_AEQE, B.Palettes(pals, dev), looks)
    if not args.no_autotune:
        log(f"autotune (tile, cut): {ctx.spl_autotune(parts, orbit[0], prm)}")
    imgs = [torch.empty((p.height, p.width, 3), dtype=torch.float32, device=dev) for p in orbit]
    prms = [prm] * len(orbit)

    def step():
        ctx.spl_render_batch(parts, orbit, prms, outs=imgs, stats=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    frames = args.steps * len(orbit)
    value = frames * ps.n / elapsed
    log(f"orbit: {frames} frames in {elapsed:.3f} s, {1e3 * elapsed / frames:.3f} ms per frame")

    rows = []
    img = torch.empty((sweep[0].height, sweep[0].width, 3), dtype=torch.float32, device=dev)
    for k, pose in enumerate(sweep):
        rec, _ = ctx.spl_project(parts, pose, prm)
        sig = rec.view(-1, 8)[:, 4]
        act = sig > 0
        mean_r = float(3.0 * sig[act].mean()) if bool(act.any()) else 0.0
        n_act = int(act.sum())
        del rec, sig, act
        ctx.spl_render(parts, pose, prm, out=img, stats=False)
        torch.cuda.synchronize()
        reps = 5
        t1 = time.perf_counter()
        for _ in range(reps):
            ctx.spl_render(parts, pose, prm, out=img, stats=False)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1) / reps
        eye = np.asarray(pose.eye) - 0.5
        rows.append({"distance": float(np.linalg.norm(eye)), "mean_radius_px": mean_r,
                     "n_active": n_act, "ms_per_frame": ms,
                     "ns_per_particle": 1e6 * ms / ps.n})
        log(f"sweep {k}: {rows[-1]}")
    out = base_record(args, value, 1e3 * elapsed / args.steps, "f32", {
        "workload": f"orbit animation: Soneira-Peebles clustered set, {ps.n} particles, 2 species, "
                    "100-frame orbit at 1024x1024 per step in one batched call, additive "
                    "absorption=emission, FP32; plus a 6-pose far-to-near sweep",
        "n_particles": ps.n, "image": [1024, 1024], "frames_per_step": len(orbit),
        "batch_workspace_gib": args.batch_gib})
    out.update({"ms_per_frame": 1e3 * elapsed / frames, "sweep": rows})
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ps, orbit[:1], looks, pals,
                                           args.cpu_sample or 2_000_000, B.SPL_ADD_AEQE)
    return out


def run_blobs(args, torch, B):
    """The small case: 100k particles in 64 Gaussian blobs at 256^2, fixed
    camera, additive absorption = emission; GPU time per frame against the
    oracle's on the same frame, and the image error."""
    from oracle import splref as R
    from paper_1606_04427_amd import synth

    ps = synth.blobs(args.n or 100_000, seed=1000)
    cam = synth.blobs_camera(256, 256)
    s_ = ps.scalar[ps.scalar > 0]
    looks = [dict(log10=1, brightness=0.3, lo=float(np.log10(s_.min())),
                  hi=float(np.log10(s_.max())))]
    pals = [synth.palette(0)]
    dev = "cuda:0"
    ctx = B.Context(0)
    parts = B.DeviceParticles(ps, dev, "f32")
    prm = B.make_params(B.SPL_ADD_AEQE, B.Palettes(pals, dev), looks)
    img = torch.empty((256, 256, 3), dtype=torch.float32, device=dev)

    def step():
        ctx.spl_render(parts, cam, prm, out=img, stats=False)

    elapsed, ms, by, frames = timed_steps(ctx, step, args.steps, args.warmup, torch)
    ms_per_step = 1e3 * elapsed / args.steps
    R.build(force=False)
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    P = R.Particles(ps)
    t0 = time.perf_counter()
    ref = R.render(P, cam, R.params(R.ADD_AEQE, L))
    dt = time.perf_counter() - t0
    got = img.cpu().numpy().astype(np.float64)
    out = base_record(args, ps.n / (ms_per_step * 1e-3), ms_per_step, "f32", {
        "workload": f"{ps.n} particles in 64 Gaussian blobs, 256x256, fixed camera, additive "
                    "absorption=emission, FP32", "n_particles": ps.n, "image": [256, 256]})
    out.update({"roofline": roofline_for(B, ms, by, frames), "stages": stage_table(B, ms, by, frames),
                "rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                "cpu_baseline": {"value": ps.n / dt, "unit": "particles/s", "cores": 1,
                                 "kind": "oracle",
                                 "sample": f"the whole frame, FP64 single-threaded C oracle, "
                                           f"{dt:.2f} s"}})
    ctx.close()
    return out


def run_sorted(args, torch, B):
    t = time.time()
    ps, poses, looks, pals = workload(args.n or 10_000_000, width=2048, height=2048,
                                      absorption=True)
    log(f"generated {ps.n} particles in {time.time() - t:.1f} s")
    dev = "cuda:0"
    ctx = B.Context(0)
    parts = B.DeviceParticles(ps, dev, "f32")
    prm = B.make_params(B.SPL_SORTED, B.Palettes(pals, dev), looks)
    pose = poses[0]
    img = torch.empty((pose.height, pose.width, 3), dtype=torch.float32, device=dev)
    tile = None
    if not args.no_autotune:
        tile, _ = ctx.spl_autotune(parts, pose, prm)
        log(f"autotune: tile {tile}")

    def step():
        ctx.spl_render(parts, pose, prm, out=img, stats=False)

    elapsed, ms, by, frames = timed_steps(ctx, step, args.steps, args.warmup, torch)
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps * ps.n / elapsed
    st = ctx.spl_render(parts, pose, prm, out=img)[1]
    rec, _ = ctx.spl_project(parts, pose, prm)
    updates, _ = box_pixels(rec.cpu().numpy(), pose.width, pose.height, 0.0)
    del rec
    log(f"{args.steps} steps in {elapsed:.3f} s, {ms_per_step:.2f} ms/step, {value:.3e} particles/s")
    out = base_record(args, value, ms_per_step, "f32", {
        "workload": "Soneira-Peebles clustered set, 10M particles with absorption U[0.01,0.5], "
                    "2048x2048, depth-sorted transfer, FP32", "n_particles": ps.n,
        "image": [2048, 2048], "poses": 1, "tile": st["tile"]})
    roof = roofline_for(B, ms, by, frames, updates, FLOPS_PER_COMPOSITE_UPDATE)
    if roof["kernel"] == "k_splat_add":
        roof["kernel"] = "k_composite"  # the sorted mode's splat stage
    out.update({"roofline": roof, "stages": stage_table(B, ms, by, frames),
                "frame": {"n_active": st["n_active"], "n_pairs": st["n_pairs"]}})
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ps, [pose], looks, pals, args.cpu_sample or ps.n,
                                           B.SPL_SORTED)
    return out


# ----------------------------------------------------------------------------
def run_batched(args, torch, B, fixed=None):
    """fixed: {image width: (tile, cut)} to use instead of tuning."""
    from oracle import splref as R
    from paper_1606_04427_amd import synth

    n = args.n or 200_000_000
    t = time.time()
    ps = synth.soneira_peebles(n, seed=1003)
    log(f"generated {ps.n} particles in {time.time() - t:.1f} s")
    big = synth.random_poses(32, seed=2003, width=4096, height=4096)
    small = synth.random_poses(32, seed=2004, width=1024, height=1024)
    poses = [p for pair in zip(big, small) for p in pair][: args.views]
    looks, pals = looks_for(ps)
    dev = "cuda:0"
    pal_d = B.Palettes(pals, dev)
    prm = B.make_params(B.SPL_ADD_AEQE, pal_d, looks)
    imgs = [torch.empty((p.height, p.width, 3), dtype=torch.float32, device=dev) for p in poses]
    rng = np.random.Generator(np.random.PCG64(11))
    sub_idx = np.sort(rng.choice(ps.n, min(ps.n, 1_000_000), replace=False))
    sub = ps.subset(sub_idx)
    results = {}
    for dt_name in args.dtypes.split(","):
        ctx = B.Context(0)
        ctx.spl_set_option(B.SPL_OPT_BATCH_BYTES, args.batch_gib << 30)
        parts = B.DeviceParticles(ps, dev, dt_name)
        torch.cuda.synchronize()
        prms = [prm] * len(poses)
        tuned, trials = {}, {}
        if fixed:
            tuned = dict(fixed)
            prms = [B.make_params(B.SPL_ADD_AEQE, pal_d, looks, tile=tuned[p.width][0],
                                  large_cut=tuned[p.width][1]) for p in poses]
        elif not args.no_autotune:
            # one tuning per image size; the library applies the latest choice
            # for an image size to the poses it did not tune
            for p in (big[0], small[0]):
                tuned[p.width] = ctx.spl_autotune(parts, p, prm)
            log(f"{dt_name} autotune (tile, cut): {tuned}")
            # the single-view timing does not see the batch (its 4096-entry
            # work items, the binning of 32 large views): each image size's
            # choice is confirmed by timing the batched call itself with each
            # candidate, the other size held at its current choice
            def batch_time(choice):
                cp = [B.make_params(B.SPL_ADD_AEQE, pal_d, looks, tile=choice[p.width][0],
                                    large_cut=choice[p.width][1]) for p in poses]
                ctx.spl_render_batch(parts, poses, cp, outs=imgs, stats=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.spl_render_batch(parts, poses, cp, outs=imgs, stats=False)
                torch.cuda.synchronize()
                return time.perf_counter() - t0

            for w, extra in ((big[0].width, [(16, -1.0), (32, -1.0)]),
                             (small[0].width, [(16, -1.0)])):
                times = {}
                for tc in sorted({tuple(tuned[w]), *extra}):
                    times[tc] = batch_time({**tuned, w: tc})
                tuned[w] = min(times, key=times.get)
                trials[w] = {f"{k[0]}/{k[1]:g}": round(v * 1e3) for k, v in times.items()}
            prms = [B.make_params(B.SPL_ADD_AEQE, pal_d, looks, tile=tuned[p.width][0],
                                  large_cut=tuned[p.width][1]) for p in poses]
            log(f"{dt_name} batched choices: {tuned} (step ms per candidate: {trials})")

        def bstep():
            ctx.spl_render_batch(parts, poses, prms, outs=imgs, stats=False)

        def gstep():
            # the same call with the launches after each list-size
            # synchronisation captured and replayed as a graph
            ctx.spl_set_option(B.SPL_OPT_GRAPHS, 1)
            try:
                ctx.spl_render_batch(parts, poses, prms, outs=imgs, stats=False)
            finally:
                ctx.spl_set_option(B.SPL_OPT_GRAPHS, 0)

        def pstep():
            for k, p in enumerate(poses):
                ctx.spl_render(parts, p, prms[k], out=imgs[k], stats=False)

        res = {}
        # stage times of one batched step (library HIP events)
        bstep()
        _, sms, sby, sfr = timed_steps(ctx, bstep, 1, 0, torch)
        res["stages_ms_per_step"] = {B.STAGES[k]: sms[k] for k in range(len(sms))}
        log(f"{dt_name} stages per step (ms): "
            + ", ".join(f"{k} {v:.1f}" for k, v in res["stages_ms_per_step"].items() if v > 0.05))
        for name, fn in (("batched", bstep), ("batched_graph", gstep), ("per_view", pstep)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[name] = {"ms_per_step": 1e3 * dt / args.steps,
                         "particles_per_s": args.steps * len(poses) * ps.n / dt}
            log(f"{dt_name} {name}: {res[name]}")
        del parts
        # error against the FP64 oracle on a fixed 1M subsample, views
        # alternating 4096^2 and 1024^2, rendered by the batched call with the
        # tile and cut the timed run used at each image size
        sparts = B.DeviceParticles(sub, dev, dt_name)
        L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
        RP = R.Particles(sub)
        errs = []
        t_err = time.time()
        eposes = poses[: args.error_views]
        eprms = []
        for p in eposes:
            tile, cut = tuned.get(p.width, (0, 0.0))
            eprms.append(B.make_params(B.SPL_ADD_AEQE, pal_d, looks, tile=tile, large_cut=cut))
        gots, _ = ctx.spl_render_batch(sparts, eposes, eprms)
        for p, g in zip(eposes, gots):
            want = R.render(RP, p, R.params(R.ADD_AEQE, L))
            got = g.cpu().numpy().astype(np.float64)
            den = np.linalg.norm(want)
            errs.append({"image": [p.width, p.height], "tile_cut": list(tuned.get(p.width, ())),
                         "rel_l2": float(np.linalg.norm(got - want) / den) if den else 0.0,
                         "max_abs": float(np.abs(got - want).max()),
                         "max_ref": float(np.abs(want).max())})
        res["error_vs_fp64_oracle_1M_subsample"] = errs
        log(f"{dt_name} error check on {len(errs)} views in {time.time() - t_err:.1f} s: "
            + ", ".join(f"{e['rel_l2']:.2e}" for e in errs))
        res["tile_cut_by_size"] = {str(k): list(v) for k, v in tuned.items()}
        res["batched_step_ms_by_choice"] = {str(k): v for k, v in trials.items()}
        results[dt_name] = res
        ctx.close()
        del sparts
        torch.cuda.empty_cache()
    first = results[args.dtypes.split(",")[0]]
    value = first["batched"]["particles_per_s"]
    out = base_record(args, value, first["batched"]["ms_per_step"], args.dtypes.split(",")[0], {
        "workload": f"Soneira-Peebles clustered set, {ps.n} particles, {len(poses)} views "
                    "alternating 4096^2 and 1024^2, additive absorption=emission, reduced-"
                    "precision attributes, batched launches", "n_particles": ps.n,
        "views": len(poses), "batch_workspace_gib": args.batch_gib})
    out["variants"] = results
    return out


# ----------------------------------------------------------------------------
def serving_experiment(args, torch, B, n, n_requests, rates, workers):
    """The request loop on a resident clustered set: image sizes uniform over
    256^2 .. 4096^2, 80% absorption = emission and 20% depth-sorted views,
    random poses and looks.  Returns the closed-loop capacity of one call per
    view, the server's closed-loop throughput, and p50/p99 latency of both
    under Poisson arrivals at each rate (a multiple of the one-call-per-view
    capacity).  Each comparison runs the same list of views through both
    paths."""
    from paper_1606_04427_amd import serve, synth

    t = time.time()
    ps = synth.soneira_peebles(n, seed=1004, absorption=True)
    log(f"serving: generated {ps.n} particles in {time.time() - t:.1f} s")
    dev = "cuda:0"
    up = B.Context(0)
    ds = B.Dataset(up, ps, "f32")
    bank = []
    for k in range(8):
        looks, pals = looks_for(ps, scale=1.0 + 0.25 * k, palette_offset=k)
        bank.append((B.Palettes(pals, dev), looks))
    del ps
    sizes = [256, 512, 1024, 2048, 4096]
    rng = np.random.Generator(np.random.PCG64(41))

    def make(count, base):
        out = []
        for k in range(count):
            s = sizes[rng.integers(len(sizes))]
            pose = synth.random_poses(1, seed=base + k, width=s, height=s)[0]
            mode = B.SPL_SORTED if rng.uniform() < 0.2 else B.SPL_ADD_AEQE
            out.append(serve.Request(base + k, pose, mode, look=int(rng.integers(8))))
        return out

    def fresh(reqs):
        """The same views (pose, size, mode, look) as new requests, so that
        the server and the plain path are timed on identical work."""
        return [serve.Request(r.rid, r.pose, r.mode, look=r.look) for r in reqs]

    cost = lambda r: serve.request_cost(ds.n, r.pose.width, r.pose.height,
                                        r.mode == B.SPL_SORTED)
    keep = lambda r: False
    result = {"n_particles": ds.n, "workers": workers, "budget_bytes": args.budget,
              "max_views": args.max_views}
    # plain path: one request per call on one stream, closed loop (capacity)
    ex = serve.GpuExecutor(ds, bank)
    warm = make(args.warm_requests, 10_000)
    for r in warm:
        r.pose.width = r.pose.height = max(sizes)
    serve.one_per_call(ex, warm, keep=keep)
    closed_set = make(n_requests, 20_000)
    cap = serve.summary(serve.one_per_call(ex, fresh(closed_set), keep=keep))
    result["one_per_call_closed_loop"] = cap
    log(f"one per call, closed loop: {cap}")
    capacity = cap["frames_per_s"]
    # each worker's batched call may use half its share of the budget for
    # per-view buffers; the rest covers its single-view (sorted) buffers,
    # list entries and the images in flight
    srv = serve.Server(lambda w: serve.GpuExecutor(ds, bank,
                                                   batch_bytes=args.budget // (2 * workers)),
                       n_workers=workers, budget_bytes=args.budget, max_views=args.max_views,
                       cost=cost, keep=keep).start()
    # warm-up: full batches of the largest views on every worker, so the
    # workspaces reach their final size before timing
    warm = make(workers * args.max_views, 30_000)
    for r in warm:
        r.pose.width = r.pose.height = max(sizes)
    serve.drive(srv, warm, np.zeros(len(warm)))
    reqs = fresh(closed_set)
    serve.drive(srv, reqs, np.zeros(len(reqs)))
    closed = serve.summary(reqs)
    closed["batches"] = srv.n_batches
    result["server_closed_loop"] = closed
    log(f"server, closed loop: {closed}")
    for frac in rates:
        rate = frac * capacity
        arr = synth.poisson_arrivals(n_requests, rate, seed=int(1000 * frac))
        views = make(n_requests, int(50_000 + 10_000 * frac))
        reqs = fresh(views)
        serve.drive(srv, reqs, arr)
        s_ = serve.summary(reqs)
        s_["offered_rate"] = rate
        result[f"server_poisson_{frac:g}x"] = s_
        log(f"server at {frac:g} x capacity: {s_}")
        b = serve.summary(serve.one_per_call(ex, fresh(views), arr, keep=keep))
        b["offered_rate"] = rate
        result[f"one_per_call_poisson_{frac:g}x"] = b
        log(f"one per call at {frac:g} x capacity: {b}")
    result["trims"] = srv.n_trims
    result["peak_accounted_bytes"] = srv.peak_reserved
    srv.stop()
    # per image size and mode: the plain path's stage times against each
    # stage's algorithmic bytes at the HBM peak (the floor no batching of
    # independent views can go below)
    floors = {}
    ctx = ex.ctx
    for size in sizes:
        pose = synth.random_poses(1, seed=70_000 + size, width=size, height=size)[0]
        for mode, name in ((B.SPL_ADD_AEQE, "additive"), (B.SPL_SORTED, "sorted")):
            prm = ex.params(mode, 0)
            ctx.spl_render_dataset(ds, pose, prm, stats=False)
            ctx.spl_set_timing(True)
            ctx.spl_get_timing()
            for _ in range(2):
                ctx.spl_render_dataset(ds, pose, prm, stats=False)
            ms, by, fr = ctx.spl_get_timing()
            ctx.spl_set_timing(False)
            fr = max(fr, 1)
            floors[f"{size}_{name}"] = {
                "frame_ms": sum(ms) / fr,
                "hbm_floor_ms": sum(by) / fr / (HBM_PEAK_GBS * 1e9) * 1e3,
                "stages_ms": {B.STAGES[k]: ms[k] / fr for k in range(len(ms))},
                "stages_floor_ms": {B.STAGES[k]: by[k] / fr / (HBM_PEAK_GBS * 1e9) * 1e3
                                    for k in range(len(ms))}}
    result["plain_path_stage_floors"] = floors
    ex.close()
    result["speedup_vs_one_per_call"] = closed["frames_per_s"] / capacity
    ds.close()
    up.close()
    return result


def serving_leg(args, torch, B):
    """The serving sub-record of the default line: 100M resident particles,
    closed-loop throughput and p50/p99 at 1.0x the one-call-per-view
    capacity."""
    torch.cuda.empty_cache()
    return serving_experiment(args, torch, B, args.serving_n, args.serving_requests, [1.0],
                              args.workers)


def run_serving(args, torch, B):
    result = serving_experiment(args, torch, B, args.n or 100_000_000, args.requests, args.rates,
                                args.workers)
    value = result["server_closed_loop"]["frames_per_s"]
    out = base_record(args, value, 1e3 / value, "f32", {
        "workload": f"serving: {result['n_particles']} resident clustered particles, views "
                    "256^2..4096^2, 80% additive / 20% depth-sorted, 8 looks",
        "n_particles": result["n_particles"], "workers": args.workers,
        "budget_bytes": args.budget, "max_views": args.max_views})
    out["unit"] = "frames/s"
    out["speedup_vs_one_per_call"] = result["speedup_vs_one_per_call"]
    out["serving"] = result
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="additive",
                    choices=["additive", "blobs", "sorted", "batched", "serving", "orbit"])
    ap.add_argument("--n", type=int, default=0, help="particles (0: the workload's size)")
    ap.add_argument("--cpu-sample", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="additive: fixed tile (no autotune)")
    ap.add_argument("--cut", type=float, default=32.0, help="additive: fixed large cut with --tile")
    ap.add_argument("--no-probe", action="store_true", help="additive: skip the bandwidth probe")
    ap.add_argument("--no-stream", action="store_true", help="additive: skip out-of-core rendering")
    ap.add_argument("--stream-chunk", type=int, default=2_500_000,
                    help="additive: particles per out-of-core chunk")
    ap.add_argument("--no-cut-table", action="store_true",
                    help="additive: skip the per-pose frame times at each large cut")
    ap.add_argument("--no-serving", action="store_true",
                    help="additive: skip the serving sub-record")
    ap.add_argument("--no-sorted-leg", action="store_true",
                    help="additive: skip the depth-sorted sub-record")
    ap.add_argument("--no-orbit-leg", action="store_true",
                    help="additive: skip the 55M-particle orbit animation sub-record")
    ap.add_argument("--no-batched-leg", action="store_true",
                    help="additive: skip the 200M-particle, 64-view BF16 batched sub-record")
    ap.add_argument("--no-deterministic-leg", action="store_true",
                    help="additive: skip the list-order (bit-identical) frames")
    ap.add_argument("--no-graph-replay", action="store_true",
                    help="additive: skip the timing of the captured-graph replay")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="additive: also run one plain device copy of this size")
    ap.add_argument("--dtypes", default="bf16,f16,f32",
                    help="batched: attribute dtypes (the first gives the value; FP32 is the comparison)")
    ap.add_argument("--views", type=int, default=64, help="batched: views per step")
    ap.add_argument("--batch-gib", type=int, default=160,
                    help="batched and orbit: GiB of per-view workspace one batched call may "
                         "hold (SPL_OPT_BATCH_BYTES; the library's default is 48): fewer, longer "
                         "persistent launches")
    ap.add_argument("--error-views", type=int, default=4, help="batched: views checked")
    ap.add_argument("--requests", type=int, default=150, help="serving: requests per run")
    ap.add_argument("--warm-requests", type=int, default=20)
    ap.add_argument("--workers", type=int, default=2,
                    help="serving: request-loop workers (contexts and streams)")
    ap.add_argument("--serving-n", type=int, default=100_000_000,
                    help="additive: particles of the serving sub-record")
    ap.add_argument("--serving-requests", type=int, default=60,
                    help="additive: requests per serving measurement")
    ap.add_argument("--max-views", type=int, default=4,
                    help="serving: views per batch (the lowest p99 of 4, 8 and 16 at 100M)")
    ap.add_argument("--budget", type=int, default=160 << 30,
                    help="serving: device bytes for images in flight and the workers' "
                         "workspace (of the 288 GB of HBM)")
    ap.add_argument("--rates", type=float, nargs="*", default=[0.5, 0.8, 1.0, 1.2])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the renderer runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1606_04427_amd import binding as B

    run = {"additive": run_additive, "blobs": run_blobs, "sorted": run_sorted,
           "batched": run_batched, "serving": run_serving, "orbit": run_orbit}[args.workload]
    out = run(args, torch, B)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
