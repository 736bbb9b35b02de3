"""Many views in one call (spl_render_batch): one list-size synchronisation for
the whole batch and one persistent splat launch over every view's work items.
Each image must equal the single-view render of the same view (both are
sums of the same FP32 contributions; the fixed-point batch sums are exact, so
only the order of the compensated folds can differ) and the FP64 oracle."""
import numpy as np
import pytest

from paper_1606_04427_amd import synth
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(oracle):
    import torch

    from paper_1606_04427_amd import binding as B

    assert torch.cuda.is_available()
    ctx = B.Context(0)
    yield B, ctx, oracle
    ctx.close()


def _setup(B, n=120_000, seed=51):
    ps = synth.soneira_peebles(n, seed=seed, absorption=True)
    looks, pals = [], []
    for k in range(2):
        s = ps.scalar[ps.species == k]
        looks.append(dict(log10=1, brightness=0.03 * (1 + k), lo=float(np.log10(s.min())),
                          hi=float(np.log10(s.max()))))
        pals.append(synth.palette(k))
    return ps, looks, pals


def _poses():
    sizes = [(256, 256), (512, 384), (200, 130), (384, 512), (256, 256), (96, 160)]
    out = []
    for k, (w, h) in enumerate(sizes):
        out += synth.random_poses(1, seed=300 + k, width=w, height=h)
    return out


@pytest.mark.parametrize("graphs", [0, 1])
def test_batch_equals_single_view_and_oracle(env, graphs):
    import torch

    B, ctx, R = env
    ps, looks, pals = _setup(B)
    parts = B.DeviceParticles(ps, "cuda:0")
    P = B.Palettes(pals)
    poses = _poses()
    modes = [1, 0, 1, 2, 1, 0]
    prms = [B.make_params(m, P, looks, tile=16, large_cut=16.0) for m in modes]
    ctx.spl_set_option(B.SPL_OPT_GRAPHS, graphs)
    outs, sts = ctx.spl_render_batch(parts, poses, prms)
    ctx.spl_set_option(B.SPL_OPT_GRAPHS, 0)
    torch.cuda.synchronize()
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    RP = R.Particles(ps)
    for pose, prm, m, o, st in zip(poses, prms, modes, outs, sts):
        single, st1 = ctx.spl_render(parts, pose, prm)
        torch.cuda.synchronize()
        got = o.cpu().numpy().astype(np.float64)
        assert rel_l2(got, single.cpu().numpy()) < 1e-6
        assert st["n_active"] == st1["n_active"] and st["n_pairs"] == st1["n_pairs"]
        ref = R.render(RP, pose, R.params(m, L))
        if np.abs(ref).max() > 0:
            assert rel_l2(got, ref) < 1e-5


def test_batch_budget_splits_launches(env):
    """A budget that holds one view forces one persistent launch per view; the
    images must not change."""
    import torch

    B, ctx, R = env
    ps, looks, pals = _setup(B, n=50_000, seed=52)
    parts = B.DeviceParticles(ps, "cuda:0")
    P = B.Palettes(pals)
    poses = _poses()[:4]
    prms = [B.make_params(1, P, looks, tile=16) for _ in poses]
    a, _ = ctx.spl_render_batch(parts, poses, prms, stats=False)
    torch.cuda.synchronize()
    a = [x.cpu().numpy() for x in a]
    ctx.spl_set_option(B.SPL_OPT_BATCH_BYTES, 1)
    b, _ = ctx.spl_render_batch(parts, poses, prms, stats=False)
    ctx.spl_set_option(B.SPL_OPT_BATCH_BYTES, 48 << 30)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert rel_l2(y.cpu().numpy(), x) < 1e-6


def test_batch_list_limit_splits_launches(env):
    """A small list-entry limit per persistent launch splits the views into
    groups that reuse the list buffers; the images must not change."""
    import torch

    B, ctx, R = env
    ps, looks, pals = _setup(B, n=50_000, seed=54)
    parts = B.DeviceParticles(ps, "cuda:0")
    P = B.Palettes(pals)
    poses = _poses()
    prms = [B.make_params(1, P, looks, tile=16, large_cut=16.0) for _ in poses]
    a, sa = ctx.spl_render_batch(parts, poses, prms)
    torch.cuda.synchronize()
    a = [x.cpu().numpy() for x in a]
    for graphs in (0, 1):
        ctx.spl_set_option(B.SPL_OPT_GRAPHS, graphs)
        ctx.spl_set_option(B.SPL_OPT_BATCH_PAIRS, 60_000)
        b, sb = ctx.spl_render_batch(parts, poses, prms)
        ctx.spl_set_option(B.SPL_OPT_BATCH_PAIRS, 0xFFFFFFFE)
        ctx.spl_set_option(B.SPL_OPT_GRAPHS, 0)
        torch.cuda.synchronize()
        for x, y, s1, s2 in zip(a, b, sa, sb):
            assert rel_l2(y.cpu().numpy(), x) < 1e-6
            assert s1["n_pairs"] == s2["n_pairs"]
    with pytest.raises(B.SplotchError):
        ctx.spl_set_option(B.SPL_OPT_BATCH_PAIRS, 0)


def test_batch_rejects_bad_view(env):
    B, ctx, _ = env
    ps, looks, pals = _setup(B, n=1000, seed=53)
    parts = B.DeviceParticles(ps, "cuda:0")
    P = B.Palettes(pals)
    poses = _poses()[:2]
    poses[1] = synth.Pose((0, 0, 1), (0, 0, 1), (0, 1, 0), 60, 0.0, 8, 8)
    prms = [B.make_params(1, P, looks) for _ in poses]
    with pytest.raises(B.SplotchError):
        ctx.spl_render_batch(parts, poses, prms)


def test_batch_with_empty_views(env):
    """A view that sees no particle (camera looking away from the set) and an
    empty particle set give black images and zero statistics in a batch."""
    import torch

    B, ctx, R = env
    ps, looks, pals = _setup(B, n=20_000, seed=55)
    parts = B.DeviceParticles(ps, "cuda:0")
    P = B.Palettes(pals)
    away = synth.Pose((0.5, 0.5, 3.0), (0.5, 0.5, 6.0), (0, 1, 0), 50.0, 0.05, 128, 96)
    poses = [away] + _poses()[:2]
    prms = [B.make_params(1, P, looks, tile=16) for _ in poses]
    outs, sts = ctx.spl_render_batch(parts, poses, prms)
    torch.cuda.synchronize()
    assert sts[0]["n_active"] == 0 and sts[0]["n_pairs"] == 0
    assert not outs[0].any().item()
    assert sts[0]["flux"] == [0.0, 0.0, 0.0]
    for o, st in zip(outs[1:], sts[1:]):
        assert st["n_active"] > 0 and o.any().item()
    empty = synth.ParticleSet(*(np.zeros(0, np.float32) for _ in range(6)), np.zeros(0, np.uint8))
    eparts = B.DeviceParticles(empty, "cuda:0")
    outs, sts = ctx.spl_render_batch(eparts, poses, prms)
    torch.cuda.synchronize()
    assert all(s["n_active"] == 0 for s in sts)
    assert not any(o.any().item() for o in outs)


@pytest.mark.parametrize("graphs", [0, 1])
def test_batch_mixed_tile_sizes(env, graphs):
    """Views asking for different tile sizes are served tile size by tile size;
    each keeps its own tile and its image and statistics equal the single-view
    render, whatever their order in the call."""
    import torch

    B, ctx, _ = env
    ps, looks, pals = _setup(B, n=60_000, seed=56)
    parts = B.DeviceParticles(ps, "cuda:0")
    P = B.Palettes(pals)
    poses = _poses()
    tiles = [32, 16, 32, 16, 16, 32]
    modes = [1, 1, 0, 2, 1, 1]
    prms = [B.make_params(m, P, looks, tile=t, large_cut=32.0) for m, t in zip(modes, tiles)]
    ctx.spl_set_option(B.SPL_OPT_GRAPHS, graphs)
    try:
        outs, sts = ctx.spl_render_batch(parts, poses, prms)
        torch.cuda.synchronize()
    finally:
        ctx.spl_set_option(B.SPL_OPT_GRAPHS, 0)
    for pose, prm, t, o, st in zip(poses, prms, tiles, outs, sts):
        single, st1 = ctx.spl_render(parts, pose, prm)
        torch.cuda.synchronize()
        assert st["tile"] == t == st1["tile"]
        assert st["n_pairs"] == st1["n_pairs"]
        assert rel_l2(o.cpu().numpy(), single.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("graphs", [0, 1])
def test_more_views_than_one_launch_serves(env, graphs):
    """150 views in one call: the batch's per-view kernels (scans, item
    builds, image clears, final maps, FP64 reductions) run in launches of up
    to 64 views, here three (64 + 64 + 22); every view, with its statistics,
    must equal its single-view render."""
    import torch

    B, ctx, R = env
    ps, looks, pals = _setup(B, n=60_000, seed=54)
    parts = B.DeviceParticles(ps, "cuda:0")
    P = B.Palettes(pals)
    sizes = [(64, 48), (96, 64), (40, 72), (128, 96), (33, 17)]
    poses = [synth.random_poses(1, seed=700 + k, width=sizes[k % 5][0],
                                height=sizes[k % 5][1])[0] for k in range(150)]
    prms = [B.make_params(1 if k % 3 else 0, P, looks, tile=16, large_cut=-1.0,
                          normalise=int(k % 7 == 0), flux_check=int(k % 11 == 0))
            for k in range(150)]
    print(f"150 views graphs={graphs}", flush=True)
    ctx.spl_set_option(B.SPL_OPT_GRAPHS, graphs)
    outs, sts = ctx.spl_render_batch(parts, poses, prms)
    ctx.spl_set_option(B.SPL_OPT_GRAPHS, 0)
    torch.cuda.synchronize()
    for k, (pose, prm, o, st) in enumerate(zip(poses, prms, outs, sts)):
        single, st1 = ctx.spl_render(parts, pose, prm)
        torch.cuda.synchronize()
        got, want = o.cpu().numpy().astype(np.float64), single.cpu().numpy().astype(np.float64)
        if np.abs(want).max() == 0:
            assert np.abs(got).max() == 0, k
            continue
        assert rel_l2(got, want) < 1e-6, k
        assert st["n_active"] == st1["n_active"] and st["n_pairs"] == st1["n_pairs"], k
        np.testing.assert_allclose(st["flux"], st1["flux"], rtol=1e-5, err_msg=str(k))
        np.testing.assert_allclose(st["max"], st1["max"], rtol=1e-5, err_msg=str(k))
        if prm.flux_check:
            np.testing.assert_allclose(st["expected_flux"], st1["expected_flux"], rtol=1e-9,
                                       err_msg=str(k))
