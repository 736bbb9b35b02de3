"""Host logic of the benchmark script, without a GPU: the roofline record of
the dominant stage, the rule that a counter profile counts only while the
kernel sources it was taken on are unchanged, the box-pixel count behind the
splat's update figure, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

import bench  # noqa: E402

STAGES = ["project", "count", "scan", "host_gap_items", "scatter", "sort", "large_splat",
          "splat", "finalise"]
B = types.SimpleNamespace(STAGES=STAGES)


def _times(**kw):
    ms = [0.0] * len(STAGES)
    by = [0.0] * len(STAGES)
    for k, (t, b) in kw.items():
        ms[STAGES.index(k)] = t
        by[STAGES.index(k)] = b
    return ms, by


def test_stage_names_match_the_library():
    from paper_1606_04427_amd import binding

    assert list(binding.STAGES) == STAGES
    for s in STAGES:
        assert s == "host_gap_items" or s in bench.KERNEL_OF_STAGE


def test_splat_dominant_is_priced_against_the_fp32_vector_peak():
    # 8 launches, 4 ms each, 1e9 updates per launch at 12 operations each
    ms, by = _times(splat=(32.0, 8 * 2e9), project=(1.0, 8 * 1e9))
    r = bench.roofline_for(B, ms, by, 8, updates_per_launch=1e9)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["peak"] == 157.3
    assert bench.FLOPS_PER_UPDATE == 12.0
    assert r["achieved"] == pytest.approx(12.0 * 1e9 / 4e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["kernel"] == "k_splat_add"
    assert r["ms_per_launch"] == pytest.approx(4.0)
    assert r["bytes_per_launch"] == pytest.approx(2e9)
    assert r["hbm_GBps"] == pytest.approx(2e9 / 4e-3 / 1e9)
    assert r["traffic"] is None


def test_composite_is_priced_with_its_own_operation_count():
    # the depth-sorted composite: 28 operations per update (the additive 12
    # plus the optical depth, the polynomial for phi, the weight and the
    # transmittance update)
    ms, by = _times(splat=(3.0, 3 * 8e8))
    r = bench.roofline_for(B, ms, by, 3, 5e8, bench.FLOPS_PER_COMPOSITE_UPDATE)
    assert bench.FLOPS_PER_COMPOSITE_UPDATE == 28.0
    assert r["bound"] == "alu" and r["flops_per_update"] == 28.0
    assert r["achieved"] == pytest.approx(28.0 * 5e8 / 1e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)


def test_other_dominant_stage_is_priced_against_hbm():
    # the host gap is never the dominant kernel, however long it is
    ms, by = _times(host_gap_items=(100.0, 0.0), scatter=(10.0, 4e10), splat=(2.0, 1e9))
    r = bench.roofline_for(B, ms, by, 5, updates_per_launch=1e9)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["kernel"] == "k_scatter"
    assert r["achieved"] == pytest.approx(4e10 / 10e-3 / 1e9)
    assert r["frac"] == pytest.approx(0.5)
    assert r["ms_per_launch"] == pytest.approx(2.0)
    assert r["bytes_per_launch"] == pytest.approx(8e9)


def test_splat_without_an_update_count_falls_back_to_bytes():
    ms, by = _times(splat=(4.0, 8e9))
    r = bench.roofline_for(B, ms, by, 1)
    assert r["bound"] == "hbm" and r["kernel"] == "k_splat_add"
    assert r["achieved"] == pytest.approx(2000.0)


def _traffic_file(tmp_path, **over):
    rec = {"kernel": "k_splat_add_views", "n": 1000, "tile": 16, "cut": -1.0,
           "sources": ["k_splat.hip", "spl_internal.h"],
           "bytes_per_launch": 12345.0}
    rec["digest"] = bench.source_digest(rec["sources"])
    rec.update(over)
    p = tmp_path / "traffic.txt"
    p.write_text("# counters\n\n```json\n" + json.dumps(rec, indent=1) + "\n```\n")
    return str(p)


def test_traffic_counts_while_the_sources_match(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path))
    assert bench.measured_traffic("k_splat_add_views", 1000, 16, -1.0) == 12345.0


@pytest.mark.parametrize("arg", [("k_splat_add", 1000, 16, -1.0),
                                 ("k_splat_add_views", 999, 16, -1.0),
                                 ("k_splat_add_views", 1000, 32, -1.0),
                                 ("k_splat_add_views", 1000, 16, 32.0)])
def test_traffic_of_another_configuration_is_not_reported(tmp_path, monkeypatch, arg):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path))
    assert bench.measured_traffic(*arg) is None


def test_traffic_taken_on_other_sources_is_not_reported(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, digest="0" * 16))
    assert bench.measured_traffic("k_splat_add_views", 1000, 16, -1.0) is None


def test_missing_or_malformed_traffic_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.txt"))
    assert bench.measured_traffic("k_splat_add_views", 1000, 16, -1.0) is None
    bad = tmp_path / "bad.txt"
    bad.write_text("no json block here\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(bad))
    assert bench.measured_traffic("k_splat_add_views", 1000, 16, -1.0) is None


def test_committed_traffic_profile_names_existing_sources():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.loads(f.read().split("```json")[1].split("```")[0])
    for n in rec["sources"]:
        assert os.path.exists(os.path.join(ROOT, "paper_1606_04427_amd", "csrc", n)), n
    assert rec["bytes_per_launch"] == pytest.approx(
        (rec["fetch_kib_per_launch_raw"] * rec["fetch_scale"]
         + rec["write_kib_per_launch_raw"] * rec["write_scale"]) * 1024.0)


def _records(rows):
    """Packed 32-byte records {Xi, Xf, Yi, Yf, sigma, r, g, b}."""
    out = np.zeros((len(rows), 8), np.float32)
    for k, (X, Y, s) in enumerate(rows):
        out[k, 0], out[k, 1] = np.floor(X), X - np.floor(X)
        out[k, 2], out[k, 3] = np.floor(Y), Y - np.floor(Y)
        out[k, 4] = s
    return out.reshape(-1)


def test_box_pixels_counts_clipped_integer_boxes():
    # sigma 1, R = 3, centre 10.25: pixel centres i + 0.5 within R of it are
    # i = 7..12, so 6 x 6
    n_px, n_small = bench.box_pixels(_records([(10.25, 10.25, 1.0)]), 64, 64, 0.0)
    assert (n_px, n_small) == (36.0, 1)
    # a centre on a pixel edge keeps both pixels at distance exactly R: 7 x 7
    n_px, _ = bench.box_pixels(_records([(10.5, 10.5, 1.0)]), 64, 64, 0.0)
    assert n_px == 49.0
    # clipped at the left and top edges: pixels 0..2 x 0..2
    n_px, _ = bench.box_pixels(_records([(0.25, 0.25, 1.0)]), 64, 64, 0.0)
    assert n_px == 9.0
    # inactive (sigma 0) records and particles above the cut do not count
    n_px, n_small = bench.box_pixels(_records([(10.25, 10.25, 1.0), (20.0, 20.0, 0.0),
                                              (30.5, 30.5, 20.0)]), 64, 64, 32.0)
    assert (n_px, n_small) == (36.0, 1)
    # a box wholly off the image covers no pixel
    n_px, _ = bench.box_pixels(_records([(80.25, 10.25, 1.0), (-9.75, -9.75, 1.0)]), 64, 64, 0.0)
    assert n_px == 0.0


def test_box_pixels_brute_force():
    rng = np.random.default_rng(5)
    rows = [(rng.uniform(-8, 72), rng.uniform(-8, 72), rng.uniform(0.2, 4.0)) for _ in range(50)]
    W, H = 64, 48
    want = 0
    for X, Y, s in rows:
        R = 3.0 * float(np.float32(s))
        # recompute the pixel centre from the stored split, as the box does
        Xs = float(np.float32(np.floor(X))) + float(np.float32(X - np.floor(X)))
        Ys = float(np.float32(np.floor(Y))) + float(np.float32(Y - np.floor(Y)))
        nx = sum(1 for i in range(W) if abs(i + 0.5 - Xs) <= R)
        ny = sum(1 for j in range(H) if abs(j + 0.5 - Ys) <= R)
        want += nx * ny
    n_px, n_small = bench.box_pixels(_records(rows), W, H, 0.0)
    assert n_small == 50
    assert n_px == want


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_record_carries_the_contract_fields():
    args = types.SimpleNamespace(steps=10, warmup=3)
    cfg = {"workload": "10M particles, 1024x1024, 8 poses", "n_particles": 10_000_000}
    r = bench.base_record(args, 1.5e10, 5.4, "f32", cfg)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in r, k
    assert r["n_gpus"] == 1 and r["steps"] == 10 and r["warmup"] == 3
    assert r["higher_is_better"] is True and r["scaling"] == "weak"
    assert r["vs_baseline"] is None and r["data"] == "synthetic"
    assert r["config"]["workload"] == cfg["workload"]
    json.dumps(r)  # one JSON line


def test_cpu_baseline_times_the_oracle_on_a_sample(oracle):
    from paper_1606_04427_amd import synth

    ps = synth.soneira_peebles(20000, seed=7)
    poses = synth.orbit_poses(2, width=64, height=64)
    looks, pals = bench.looks_for(ps)
    r = bench.cpu_baseline(ps, poses, looks, pals, 5000, 1)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "particles/s"
    assert r["value"] > 0 and "5000-particle" in r["sample"]


def test_box_pixels_agrees_with_the_oracle_box_rule(oracle):
    """The update count behind the splat's roofline uses the same pixel box
    as the binning rule (the oracle's FP32 record box), up to rounding at
    box edges."""
    rng = np.random.default_rng(11)
    W, H = 96, 80
    rows = [(rng.uniform(-10, 106), rng.uniform(-10, 90), rng.uniform(0.3, 6.0))
            for _ in range(400)]
    rec = _records(rows)
    n_px, _ = bench.box_pixels(rec, W, H, 0.0)
    want = 0
    for r in rec.reshape(-1, 8):
        ok, (i0, i1, j0, j1) = oracle.record_box(r, 3.0, W, H)
        if ok:
            want += (i1 - i0 + 1) * (j1 - j0 + 1)
    assert want > 0
    assert abs(n_px - want) <= 1e-3 * want


def test_footprint_is_the_mean_over_particle_view_pairs():
    """Two views: 3 small particles with boxes of 9, 25 and 49 px in the first,
    one of 100 px in the second; the mean is 183 / 4, whatever the number of
    views (the sums already cover every view)."""
    rec = np.zeros((4, 8), np.float32)
    # X = 50.5, Y = 50.5 (integer part + fraction), sigma chosen so R = 3 sigma
    # gives odd box widths 3, 5, 7 and 10 px
    rec[:, 0] = 50.0
    rec[:, 1] = 0.5
    rec[:, 2] = 50.0
    rec[:, 3] = 0.5
    rec[:, 4] = [0.5, 2.0 / 3.0 + 1e-4, 1.0 + 1e-4, 5.0 / 3.0]
    u1, s1 = bench.box_pixels(rec[:3], 100, 100, -1.0)
    assert (u1, s1) == (9 + 25 + 49, 3)
    rec2 = rec[3:].copy()
    rec2[:, 1] = 0.0  # X = 50.0: centres within 5 px are 45.5 .. 54.5 -> 10 columns
    rec2[:, 3] = 0.0
    u2, s2 = bench.box_pixels(rec2, 100, 100, -1.0)
    assert (u2, s2) == (100, 1)
    assert bench.footprint([u1, u2], [s1, s2]) == pytest.approx(183.0 / 4.0)


def test_radius_range_inverts_the_kernel_width():
    rho = np.array([0.0, 3.0, 30.0, 300.0])
    sig = np.sqrt((rho / 3.0) ** 2 + 0.25)
    rec = np.zeros((5, 8), np.float32)
    rec[:4, 4] = sig
    r = bench.radius_range(rec)  # the inactive record (sigma = 0) is skipped
    assert r["min"] == pytest.approx(0.0, abs=2e-3)
    assert r["max"] == pytest.approx(300.0, rel=1e-5)
    assert bench.radius_range(np.zeros((2, 8), np.float32)) is None
