"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Levels:
  P0  binning: counts and offsets bit-identical to the oracle's single-precision
      rule on the same records; each tile's list equal as a set (additive) or
      in order (depth-sorted lists, whose (depth, index) keys are unique).
  P1  render from the GPU's own records vs the oracle on the same records:
      rel-L2 <= 1e-6 (the only differences are FP32 arithmetic and kernel-edge
      decisions at the rounding level).
  P2  end to end from world inputs vs the FP64 oracle: rel-L2 <= 1e-5 and
      |diff| <= 1e-3 |ref| + 1e-5 max|ref| per pixel.
"""
import math

import numpy as np
import pytest

from paper_1606_04427_amd import synth
from tests.helpers import particles, rel_l2

pytestmark = pytest.mark.gpu

P1_TOL = 1e-6
P2_TOL = 1e-5


@pytest.fixture(scope="module")
def env(oracle):
    import torch

    from paper_1606_04427_amd import binding as B

    assert torch.cuda.is_available(), "GPU tests need a device"
    ctx = B.Context(0)
    yield B, ctx, oracle
    ctx.close()


def _looks(ps, n_species=1, brightness=0.3, log10=True):
    looks, pals = [], []
    for k in range(n_species):
        s = ps.scalar[ps.species == k] if n_species > 1 else ps.scalar
        s = s[s > 0] if log10 else s
        lo = float(np.log10(s.min())) if (log10 and s.size) else (float(s.min()) if s.size else 0.0)
        hi = float(np.log10(s.max())) if (log10 and s.size) else (float(s.max()) if s.size else 1.0)
        looks.append(dict(log10=int(log10), brightness=brightness * (1 + k), lo=lo, hi=max(hi, lo)))
        pals.append(synth.palette(k))
    return looks, pals


def _gpu(env, ps, pose, mode, looks, pals, stats=False, **kw):
    import torch

    B, ctx, _ = env
    parts = B.DeviceParticles(ps, "cuda:0", kw.pop("attr_dtype", "f32"))
    prm = B.make_params(mode, B.Palettes(pals), looks, **kw)
    img, st = ctx.spl_render(parts, pose, prm)
    torch.cuda.synchronize()
    out = img.cpu().numpy().astype(np.float64)
    return (out, st) if stats else out


def _ref(env, ps, pose, mode, looks, pals, **kw):
    _, _, R = env
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    kw = {k: v for k, v in kw.items() if k in ("k_sigma", "sigma_min", "nu", "normalise")}
    return R.render(R.Particles(ps), pose, R.params(mode, L, **kw))


def _check_p2(got, ref, tol=P2_TOL, what=""):
    e = rel_l2(got, ref)
    assert e <= tol, f"{what}: rel-L2 {e:.3e} > {tol:.1e}"
    bound = 1e-3 * np.abs(ref) + 1e-5 * np.abs(ref).max()
    bad = np.abs(got - ref) > bound
    assert not bad.any(), f"{what}: {int(bad.sum())} pixels outside the max-pixel bound"
    return e


def _blob_case(n=20000, W=256, H=256, seed=21):
    ps = synth.blobs(n, seed=seed)
    return ps, synth.blobs_camera(W, H)


def _sp_case(n=60000, W=256, H=256, seed=31, pose_seed=41, absorption=False):
    ps = synth.soneira_peebles(n, seed=seed, absorption=absorption)
    poses = synth.random_poses(4, seed=pose_seed, width=W, height=H)
    return ps, poses


# ---------------------------------------------------------------- P2 end to end

@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("tile", [16, 32])
def test_blobs_end_to_end(env, mode, tile):
    ps, cam = _blob_case()
    if mode == 2:
        ps.absorption = np.random.Generator(np.random.PCG64(3)).uniform(0.01, 0.5, ps.n).astype(np.float32)
    looks, pals = _looks(ps)
    got, st = _gpu(env, ps, cam, mode, looks, pals, stats=True, tile=tile)
    ref = _ref(env, ps, cam, mode, looks, pals)
    _check_p2(got, ref, what=f"mode {mode} tile {tile}")
    _, _, R = env
    flux, mx = R.image_stats(ref)
    np.testing.assert_allclose(st["flux"], flux, rtol=1e-5)
    np.testing.assert_allclose(st["max"], mx, rtol=1e-5)


@pytest.mark.parametrize("W,H", [(100, 70), (33, 257), (1, 1), (17, 16)])
def test_ragged_image_sizes(env, W, H):
    ps, _ = _blob_case(4000, seed=22)
    cam = synth.blobs_camera(W, H)
    looks, pals = _looks(ps)
    for mode in (0, 2):
        if mode == 2:
            ps.absorption = np.full(ps.n, 0.2, np.float32)
        got = _gpu(env, ps, cam, mode, looks, pals)
        ref = _ref(env, ps, cam, mode, looks, pals)
        if np.abs(ref).max() == 0:
            assert np.abs(got).max() == 0
        else:
            _check_p2(got, ref, what=f"{W}x{H} mode {mode}")


@pytest.mark.parametrize("cut", [0.0, 8.0, -1.0])
def test_clustered_close_poses_large_path(env, cut):
    """Soneira-Peebles set seen from inside and outside the cube: kernel radii
    span sub-pixel to hundreds of px, so the large-particle path (cut 8 px
    forces most of them onto it; -1 disables it) must agree with the oracle."""
    ps, poses = _sp_case()
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    for k, pose in enumerate(poses):
        got, st = _gpu(env, ps, pose, 1, looks, pals, stats=True, large_cut=cut)
        ref = _ref(env, ps, pose, 1, looks, pals)
        if cut == 8.0 and k == 0:
            assert st["n_large"] > 0
        if np.abs(ref).max() > 0:
            _check_p2(got, ref, what=f"pose {k} cut {cut}")


def test_sorted_clustered(env):
    ps, poses = _sp_case(absorption=True)
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    for k, pose in enumerate(poses[:3]):
        got = _gpu(env, ps, pose, 2, looks, pals)
        ref = _ref(env, ps, pose, 2, looks, pals)
        if np.abs(ref).max() > 0:
            _check_p2(got, ref, what=f"sorted pose {k}")


def test_dense_tile_multi_chunk(env):
    """Thousands of particles inside one tile: the list splits into many work
    items (atomic merge for additive, ordered partial merge for sorted) and
    the sorted lists need merge passes beyond the in-LDS chunk sort."""
    rng = np.random.Generator(np.random.PCG64(5))
    n = 30000
    pts = rng.normal(0.0, 0.004, size=(n, 3))
    ps = particles(pts, h=rng.uniform(0.001, 0.02, n), intensity=rng.lognormal(0, 0.5, n),
                   scalar=rng.uniform(0.5, 2.0, n), absorption=rng.uniform(0.01, 0.5, n))
    cam = synth.Pose((0.0, 0.0, 3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 1e-3, 128, 96)
    looks, pals = _looks(ps, brightness=0.01)
    for mode in (0, 1, 2):
        got = _gpu(env, ps, cam, mode, looks, pals, tile=16)
        ref = _ref(env, ps, cam, mode, looks, pals)
        _check_p2(got, ref, what=f"dense mode {mode}")


def test_sorted_is_deterministic(env):
    ps, poses = _sp_case(30000, absorption=True)
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    a = _gpu(env, ps, poses[1], 2, looks, pals)
    b = _gpu(env, ps, poses[1], 2, looks, pals)
    assert np.array_equal(a, b)


def test_empty_and_fully_clipped(env):
    _, cam = _blob_case()
    looks = [dict(log10=0, brightness=1.0, lo=0.0, hi=1.0)]
    pals = [synth.palette(0)]
    empty = particles(np.zeros((0, 3)), h=np.zeros(0), absorption=np.zeros(0))
    for mode in (0, 1, 2):
        got, st = _gpu(env, empty, cam, mode, looks, pals, stats=True)
        assert not got.any() and st["n_active"] == 0
    behind = particles([[0.5, 0.5, 5.0], [0.5, 0.5, 3.0]], h=0.1, absorption=[0.1, 0.1])
    got, st = _gpu(env, behind, cam, 0, looks, pals, stats=True)
    assert not got.any() and st["n_active"] == 0


def test_single_particle_covering_the_image(env):
    """One particle far larger than the image (large path, every large tile)."""
    ps = particles([[0.5, 0.5, 0.5]], h=0.6, intensity=1.0, scalar=0.5)
    cam = synth.blobs_camera(192, 160)
    looks, pals = _looks(ps, log10=False)
    looks[0].update(lo=0.0, hi=1.0)
    for cut in (8.0, -1.0):
        got, st = _gpu(env, ps, cam, 0, looks, pals, stats=True, large_cut=cut)
        ref = _ref(env, ps, cam, 0, looks, pals)
        _check_p2(got, ref, what=f"cut {cut}")
        assert st["n_large"] == (1 if cut > 0 else 0)


def test_normalise_and_nu(env):
    ps, cam = _blob_case(8000, seed=23)
    looks, pals = _looks(ps)
    for kw in (dict(normalise=1), dict(nu=2.0), dict(nu=4.5, sigma_min=0.7, k_sigma=0.5)):
        got = _gpu(env, ps, cam, 0, looks, pals, **kw)
        ref = _ref(env, ps, cam, 0, looks, pals, **kw)
        _check_p2(got, ref, what=str(kw))


def test_scalar_range_matches_oracle(env):
    B, ctx, R = env
    ps, _ = _sp_case(20000)
    ps.scalar[:5] = [-1.0, 0.0, np.inf, np.nan, 1e-30]
    parts = B.DeviceParticles(ps, "cuda:0")
    for log10 in (0, 1):
        lo, hi = ctx.spl_scalar_range(parts, 2, bool(log10))
        rlo, rhi = R.scalar_range(R.Particles(ps), 2, log10)
        np.testing.assert_allclose(lo, rlo, rtol=1e-15)
        np.testing.assert_allclose(hi, rhi, rtol=1e-15)


# ---------------------------------------------------------------- P0 / P1 on records

def _records(env, ps, pose, mode, looks, pals, **kw):
    import torch

    B, ctx, _ = env
    parts = B.DeviceParticles(ps, "cuda:0")
    prm = B.make_params(mode, B.Palettes(pals), looks, **kw)
    rec, rec2 = ctx.spl_project(parts, pose, prm, with_rec2=True)
    torch.cuda.synchronize()
    return rec, rec2, prm


def test_records_match_oracle_projection(env):
    ps, poses = _sp_case(30000, absorption=True)
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    _, _, R = env
    for pose in poses[:2]:
        rec, rec2, _ = _records(env, ps, pose, 2, looks, pals)
        rec, rec2 = rec.cpu().numpy(), rec2.cpu().numpy()
        L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
        pr = R.project(R.Particles(ps), pose, R.params(2, L))
        act_r = np.array([o.active for o in pr], bool)
        act_g = rec[:, 4] > 0
        # activeness may differ only where a pixel box edge sits on a rounding boundary
        assert (act_r != act_g).sum() <= 2
        both = np.nonzero(act_r & act_g)[0]
        X = np.array([pr[k].X for k in both])
        Y = np.array([pr[k].Y for k in both])
        sg = np.array([pr[k].sigma for k in both])
        Xg = rec[both, 0].astype(np.float64) + rec[both, 1]
        Yg = rec[both, 2].astype(np.float64) + rec[both, 3]
        assert np.max(np.abs(Xg - X)) < 1e-6 and np.max(np.abs(Yg - Y)) < 1e-6
        np.testing.assert_allclose(rec[both, 4], sg, rtol=1e-7)
        amp = 1.0 / (math.pi * sg ** 2)
        E = np.array([pr[k].E[:] for k in both])
        # single-precision colour lookup: the normalised scalar t carries an
        # absolute error of ~1e-7 (log10f, one multiply), which moves the
        # colour by up to that times the palette's steepest slope; on top of
        # that, about eight single-precision roundings in the interpolation
        # and the products (brightness x intensity x colour x amplitude)
        want = E * amp[:, None]
        sp = ps.species[both]
        slope = np.array([np.abs(np.diff(p.astype(np.float64), axis=0)).max(0) * (len(p) - 1)
                          for p in pals])[sp]
        bi = np.array([looks[k]["brightness"] for k in range(2)])[sp] * ps.intensity[both]
        allowed = 1e-6 * np.abs(want) + 2e-7 * (bi * amp)[:, None] * slope
        err = np.abs(rec[both, 5:8] - want)
        assert np.all(err <= allowed), f"worst excess {np.max(err / allowed):.2f}x"
        np.testing.assert_allclose(rec2[both, 1], [pr[k].zv for k in both], rtol=1e-7)


@pytest.mark.parametrize("tile", [1, 7, 16, 32, 64])
@pytest.mark.parametrize("rule", [0, 1])
def test_binning_bit_exact(env, tile, rule):
    B, ctx, R = env
    ps, poses = _sp_case(30000, absorption=True)
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    W, H = poses[0].width, poses[0].height
    rec, rec2, _ = _records(env, ps, poses[0], 2, looks, pals)
    for by_depth in (False, True):
        c, o, p = ctx.spl_bin(rec, rec2, W, H, tile, 3.0, rule, by_depth)
        c, o, p = c.cpu().numpy().view(np.uint32), o.cpu().numpy().view(np.uint32), p.cpu().numpy().view(np.uint32)
        rc, ro, rp = R.bin_records(rec.cpu().numpy(), rec2.cpu().numpy(), W, H, tile, 3.0, rule, by_depth)
        assert np.array_equal(c, rc) and np.array_equal(o, ro)
        if by_depth:
            assert np.array_equal(p, rp)
        else:
            for t in np.nonzero(rc)[0][:: max(1, len(rc) // 500)]:
                assert np.array_equal(np.sort(p[o[t]:o[t + 1]]), np.sort(rp[ro[t]:ro[t + 1]]))
            assert np.array_equal(np.sort(p), np.sort(rp))


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("rule", [0, 1])
def test_binning_bit_exact_in_windows(env, tile, rule):
    """More bins than one workgroup's LDS holds: at 512 x 384, 1 px tiles give
    196608 bins (the count in three windows of packed bins, the scatter in
    five windows with the per-unit band masks), 2 px tiles 49152 (the scatter
    in two windows, no masks)."""
    B, ctx, R = env
    ps, poses = _sp_case(30000, W=512, H=384, absorption=True)
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    W, H = poses[0].width, poses[0].height
    rec, rec2, _ = _records(env, ps, poses[0], 2, looks, pals)
    for by_depth in (False, True):
        c, o, p = ctx.spl_bin(rec, rec2, W, H, tile, 3.0, rule, by_depth)
        c, o, p = c.cpu().numpy().view(np.uint32), o.cpu().numpy().view(np.uint32), p.cpu().numpy().view(np.uint32)
        rc, ro, rp = R.bin_records(rec.cpu().numpy(), rec2.cpu().numpy(), W, H, tile, 3.0, rule, by_depth)
        assert np.array_equal(c, rc) and np.array_equal(o, ro)
        if by_depth:
            assert np.array_equal(p, rp)
        else:
            t = np.repeat(np.arange(len(rc), dtype=np.uint64), rc.astype(np.int64)) << np.uint64(32)
            assert np.array_equal(np.sort(t | p.astype(np.uint64)), np.sort(t | rp.astype(np.uint64)))


@pytest.mark.parametrize("W,H", [(128, 64), (2731, 3), (128, 128), (145, 113), (256, 128),
                                 (331, 99), (256, 160), (6827, 6), (320, 256), (3901, 21)])
def test_binning_bit_exact_at_window_limits(env, W, H):
    """1 px tiles on both sides of each limit of the binning's launch shapes:
    8192 bins (the count's packed bins from here), 16384 (one 64 KB scatter
    window), 32768 (one 64 KB window of packed count bins), 40960 (one scatter
    window in the CU's whole LDS) and 81920 (one such window of packed count
    bins; one bin more and the scatter takes three windows and the per-unit
    band masks)."""
    B, ctx, R = env
    ps, poses = _sp_case(30000, W=W, H=H, absorption=True)
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    rec, rec2, _ = _records(env, ps, poses[0], 2, looks, pals)
    for by_depth in (False, True):
        c, o, p = ctx.spl_bin(rec, rec2, W, H, 1, 3.0, 0, by_depth)
        c, o, p = c.cpu().numpy().view(np.uint32), o.cpu().numpy().view(np.uint32), p.cpu().numpy().view(np.uint32)
        rc, ro, rp = R.bin_records(rec.cpu().numpy(), rec2.cpu().numpy(), W, H, 1, 3.0, 0, by_depth)
        assert len(c) == W * H
        assert np.array_equal(c, rc) and np.array_equal(o, ro)
        if by_depth:
            assert np.array_equal(p, rp)
        else:
            t = np.repeat(np.arange(len(rc), dtype=np.uint64), rc.astype(np.int64)) << np.uint64(32)
            assert np.array_equal(np.sort(t | p.astype(np.uint64)), np.sort(t | rp.astype(np.uint64)))


def test_paper_rule_hand_case_on_device(env):
    import json
    import os

    import torch

    B, ctx, _ = env
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tile_inclusion.json")))
    X, Y, s = g["particle"]["X"], g["particle"]["Y"], g["particle"]["sigma"]
    rec = torch.tensor([[math.floor(X), X - math.floor(X), math.floor(Y), Y - math.floor(Y), s, 1, 1, 1]],
                       dtype=torch.float32, device="cuda:0")
    for rule, key in ((1, "tiles_paper_rule"), (0, "tiles_exact_box")):
        c, _, _ = ctx.spl_bin(rec, None, g["image"][0], g["image"][1], g["tile"], g["nu"], rule)
        assert np.nonzero(c.cpu().numpy())[0].tolist() == g[key]


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("tile,cut", [(16, 0.0), (32, 0.0), (16, 8.0), (32, -1.0)])
def test_render_records_matched_input(env, mode, tile, cut):
    """P1: the splat / composite / finalise stages alone."""
    import torch

    B, ctx, R = env
    ps, poses = _sp_case(40000, absorption=True)
    looks, pals = _looks(ps, n_species=2, brightness=0.05)
    pose = poses[0]
    rec, rec2, prm = _records(env, ps, pose, mode, looks, pals, tile=tile, large_cut=cut)
    img, st = ctx.spl_render_records(rec, rec2, pose, prm)
    torch.cuda.synchronize()
    got = img.cpu().numpy().astype(np.float64)
    ref = R.render_records(rec.cpu().numpy(), rec2.cpu().numpy(), pose.width, pose.height, mode)
    e = rel_l2(got, ref)
    assert e <= P1_TOL, f"rel-L2 {e:.3e}"


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("tile", [16, 32])
def test_discs_that_just_reach_a_micro_tile(env, tile, mode):
    """Hand-made records whose truncation disc reaches a neighbouring 4 x 4
    pixel block only at one pixel centre, a hair inside the radius (plus
    twins a hair outside): the splat lists an entry on a block only if its
    disc can reach one of the block's pixel centres, so a test that is too
    tight would lose exactly these edge pixels (additive splat and
    depth-sorted composite).  Every pixel is compared with the FP64 oracle
    on the same records."""
    import torch

    B, ctx, R = env
    W = H = 4 * tile
    rows = []
    k = 0
    cases = [(f, dg) for f in (1 - 1e-5, 1 - 1e-4) for dg in (True, False)] + [(1 + 1e-4, True)]
    for sig in (0.5, 1.0, 2.3):
        r = 3.0 * sig
        for frac, diag in cases:
                ox, oy = tile * (k % 4), tile * ((k // 4) % 4)
                k += 1
                d = r * frac
                # the target pixel centre, (ox + 4.5, oy + 4.5) diagonally or
                # (ox + 4.5, oy + 2.5) sideways, is the first of the block to
                # the right; the sideways particle sits a quarter pixel off
                # the pixel rows so that no other pixel centre lies at the
                # radius by accident
                if diag:
                    X = Y = 4.5 - d / np.sqrt(2.0)
                else:
                    X, Y = 4.5 - np.sqrt(d * d - 0.0625), 2.75
                X, Y = ox + X, oy + Y
                xi, yi = np.floor(X), np.floor(Y)
                rows.append([xi, X - xi, yi, Y - yi, sig, 1.0, 0.5, 0.25])
    rec_h = np.asarray(rows, np.float32)
    assert len(rows) <= 16
    rec = torch.from_numpy(rec_h).to("cuda:0")
    # sorted mode: a / (pi sigma^2) and a distinct depth per particle
    rec2_h = np.asarray([[0.3, 1.0 + 0.1 * i] for i in range(len(rows))], np.float32)
    rec2 = torch.from_numpy(rec2_h).to("cuda:0") if mode == 2 else None
    pose = synth.Pose((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), (0, 1, 0), 40.0, 1e-3, W, H)
    prm = B.make_params(mode, B.Palettes([synth.palette(0)]),
                        [dict(log10=0, brightness=1.0, lo=0.0, hi=1.0)], tile=tile,
                        large_cut=-1.0)
    img, _ = ctx.spl_render_records(rec, rec2, pose, prm)
    torch.cuda.synchronize()
    got = img.cpu().numpy().astype(np.float64)
    ref = R.render_records(rec_h, rec2_h if mode == 2 else None, W, H, mode)
    # the weakest kept contribution (record amplitudes are premultiplied;
    # the sorted transfer takes them at a transmission close to 1); the
    # slack covers the fixed-point quantum of a batch (~2^-30 of the summed
    # amplitudes), far below one lost edge contribution
    edge = np.exp(-9.0) * 0.25
    assert np.abs(ref).max() > 0
    err = np.abs(got - ref)
    assert np.all(err <= 1e-5 * np.abs(ref) + 1e-2 * edge), float(err.max())


def test_paper_bin_rule_render(env):
    """bin_rule 1 drops the corner overlaps the paper calls negligible: the
    image differs from the exact one only by those dropped contributions."""
    ps, cam = _blob_case(20000, seed=24)
    looks, pals = _looks(ps)
    exact = _gpu(env, ps, cam, 0, looks, pals, bin_rule=0)
    paper = _gpu(env, ps, cam, 0, looks, pals, bin_rule=1)
    # the splat sums in fixed point with a quantum of ~1e-7 of a batch's
    # amplitude sum, so the comparison allows that much absolute slack
    assert np.all(paper <= exact * (1 + 1e-5) + 1e-6 * exact.max())
    assert 0 < rel_l2(paper, exact) < 0.05


# ---------------------------------------------------------------- errors

def test_invalid_arguments_are_rejected(env):
    B, ctx, _ = env
    ps, cam = _blob_case(100)
    looks, pals = _looks(ps)
    parts = B.DeviceParticles(ps, "cuda:0")
    prm = B.make_params(0, B.Palettes(pals), looks)
    bad = [synth.Pose((0, 0, 1), (0, 0, 1), (0, 1, 0), 60, 0.0, 8, 8),
           synth.Pose((0, 0, 1), (0, 0, 0), (0, 0, 1), 60, 0.0, 8, 8),
           synth.Pose((0, 0, 1), (0, 0, 0), (0, 1, 0), 180.0, 0.0, 8, 8),
           synth.Pose((0, 0, 1), (0, 0, 0), (0, 1, 0), 60, 0.0, 0, 8)]
    for pose in bad:
        with pytest.raises(B.SplotchError) as ei:
            ctx.spl_render(parts, pose, prm)
        assert ei.value.status == B.SPL_EINVAL
    prm.tile = 12
    with pytest.raises(B.SplotchError):
        ctx.spl_render(parts, cam, prm)
    prm.tile = 0
    prm.mode = 2  # sorted without absorption
    with pytest.raises(B.SplotchError):
        ctx.spl_render(parts, cam, prm)


# ---------------------------------------------------------------- reduced precision

@pytest.mark.parametrize("dtype,tol", [("bf16", 2e-3), ("f16", 5e-4)])
def test_reduced_precision_attributes(env, dtype, tol):
    """Smoothing length, intensity and colour scalar stored in BF16 / FP16
    (positions stay FP32), accumulation in FP32: image error against the FP64
    oracle run on the original FP32 attributes.  BF16 keeps 8 mantissa bits
    (relative rounding 2^-9), FP16 11 bits (2^-12); per particle the error is
    a few times that, and it averages down over overlapping particles."""
    ps, poses = _sp_case(200_000, W=384, H=320)
    looks, pals = _looks(ps, n_species=2, brightness=0.02)
    errs = []
    for pose in poses[:3]:
        got = _gpu(env, ps, pose, 1, looks, pals, attr_dtype=dtype)
        ref = _ref(env, ps, pose, 1, looks, pals)
        if np.abs(ref).max() == 0:
            continue
        errs.append(rel_l2(got, ref))
        full = _gpu(env, ps, pose, 1, looks, pals)
        assert rel_l2(full, ref) <= P2_TOL
    assert errs and max(errs) <= tol, f"{dtype}: rel-L2 {errs}"
