"""The no-allocation entry point (spl_render_noalloc) against spl_render and the
FP64 oracle, through the C ABI: two calls in a row on one context, the second
with fewer particles and a smaller image, so that the second finds the first
call's contents in the shared scratch array.  The context's own workspace
must stay empty (the call allocates nothing), and frames too large for the
scratch are refused with SPL_ENOMEM."""
import ctypes as C

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
    yield B, oracle


def _looks(ps):
    looks, pals = [], []
    for k in range(2):
        s = ps.scalar[ps.species == k]
        looks.append(dict(log10=1, brightness=0.03 * (1 + k), lo=float(np.log10(s.min())),
                          hi=float(np.log10(s.max()))))
        pals.append(synth.palette(k))
    return looks, pals


@pytest.mark.parametrize("mode", [1, 0, 2])
def test_noalloc_equals_render_on_two_calls(env, mode):
    import torch

    B, R = env
    ctx = B.Context(0)
    cases = [(300_000, 61, 512, 384, 401), (100_000, 62, 256, 200, 402)]
    for n, seed, w, h, pseed in cases:
        print(f"noalloc mode={mode} n={n} image={w}x{h} seed={seed}", flush=True)
        ps = synth.soneira_peebles(n, seed=seed, absorption=True)
        looks, pals = _looks(ps)
        parts = B.DeviceParticles(ps, "cuda:0")
        P = B.Palettes(pals)
        prm = B.make_params(mode, P, looks, tile=16)
        pose = synth.random_poses(1, seed=pseed, width=w, height=h)[0]
        got, st = ctx.spl_render_noalloc(parts, pose, prm)
        torch.cuda.synchronize()
        assert ctx.workspace_bytes() == 0  # nothing allocated by the context
        g = got.cpu().numpy().astype(np.float64)
        ref_gpu, st1 = ctx.spl_render(parts, pose, prm)
        torch.cuda.synchronize()
        r = ref_gpu.cpu().numpy().astype(np.float64)
        assert st["n_active"] == st1["n_active"] and st["n_pairs"] == st1["n_pairs"]
        assert st["n_active"] > 0
        if mode == 2:
            # depth-sorted compositing is deterministic: the same bits
            assert np.array_equal(g, r)
        else:
            assert rel_l2(g, r) < 1e-6
        L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
        want = R.render(R.Particles(ps), pose, R.params(mode, L))
        assert rel_l2(g, want) < 1e-5
        np.testing.assert_allclose(st["flux"], R.image_stats(g)[0], rtol=1e-9)
        # the next case starts from a context whose workspace is grown; the
        # scratch path must still leave it alone
        ctx.close()
        ctx = B.Context(0)
    ctx.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_noalloc_with_binning_in_windows(env, mode):
    """16 px tiles at 8192 x 3072 (98304 fine bins and 6144 large-particle
    bins): more bins than the CU's LDS holds, so the count runs in two
    windows and the scatter in three with the per-unit band masks, whose
    buffer the no-allocation call also takes from the scratch and gives
    back."""
    import torch

    B, R = env
    ctx = B.Context(0)
    ps = synth.soneira_peebles(200_000, seed=63, absorption=True)
    looks, pals = _looks(ps)
    parts = B.DeviceParticles(ps, "cuda:0")
    prm = B.make_params(mode, B.Palettes(pals), looks, tile=16)
    pose = synth.random_poses(1, seed=403, width=8192, height=3072)[0]
    print(f"noalloc windows mode={mode}", flush=True)
    got, st = ctx.spl_render_noalloc(parts, pose, prm)
    torch.cuda.synchronize()
    assert ctx.workspace_bytes() == 0
    ref, st1 = ctx.spl_render(parts, pose, prm)
    torch.cuda.synchronize()
    g, r = got.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64)
    assert st["n_pairs"] == st1["n_pairs"] and st["n_active"] > 0
    if mode == 2:
        assert np.array_equal(g, r)
    else:
        assert rel_l2(g, r) < 1e-6
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    assert rel_l2(g, R.render(R.Particles(ps), pose, R.params(mode, L))) < 1e-5
    ctx.close()


def _raw_particles(B, n, h_value):
    """n particles in a thin sheet in front of the camera, all arrays on the
    device; returns the struct and the tensors that keep it alive."""
    import torch

    g = torch.Generator(device="cpu").manual_seed(5)
    x = torch.rand(n, generator=g).cuda()
    y = torch.rand(n, generator=g).cuda()
    z = torch.full((n,), 0.5).cuda()
    h = torch.full((n,), float(h_value)).cuda()
    i = torch.ones(n).cuda()
    s = torch.full((n,), 0.5).cuda()
    st = B.spl_particles()
    st.n = n
    st.x, st.y, st.z = x.data_ptr(), y.data_ptr(), z.data_ptr()
    st.h, st.intensity, st.scalar = h.data_ptr(), i.data_ptr(), s.data_ptr()
    st.attr_dtype = B.SPL_F32
    st.h_scale = st.i_scale = st.s_scale = 1.0
    st.species = None
    st.absorption = None
    return st, (x, y, z, h, i, s)


def test_noalloc_refuses_frames_beyond_the_scratch(env):
    import torch

    B, _ = env
    L = B.lib()
    cap = int(L.spl_noalloc_scratch_bytes())
    assert cap == 128 << 20
    ctx = B.Context(0)
    P = B.Palettes([np.ones((1, 3), np.float32)])
    prm = B.make_params(1, P, [dict(log10=0, brightness=1.0, lo=0.0, hi=1.0)], tile=16,
                        large_cut=-1.0)
    pose = synth.Pose((0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 40.0, 1e-3, 256, 256)
    out = torch.zeros((256, 256, 3), device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    cam = B.make_camera(pose)
    # too many particles for the per-particle buffers: refused before any work
    n_big = cap // 40 + 1000
    print(f"noalloc refusal: n={n_big}", flush=True)
    st, keep = _raw_particles(B, n_big, 1e-3)
    rc = L.spl_render_noalloc(ctx.h, C.byref(st), C.byref(cam), C.byref(prm),
                              C.c_void_p(out.data_ptr()), None, stream)
    assert rc == B.SPL_ENOMEM
    assert b"scratch" in L.spl_last_error(ctx.h)
    del keep
    # few particles but tile lists too long for what is left: refused after
    # the count (boxes of about 94 px: some 40 tiles per particle, 128 MB of
    # list entries)
    n_mid = 800_000
    print(f"noalloc refusal after the count: n={n_mid}", flush=True)
    st, keep = _raw_particles(B, n_mid, 0.2)
    rc = L.spl_render_noalloc(ctx.h, C.byref(st), C.byref(cam), C.byref(prm),
                              C.c_void_p(out.data_ptr()), None, stream)
    assert rc == B.SPL_ENOMEM
    assert b"scratch" in L.spl_last_error(ctx.h)
    torch.cuda.synchronize()
    del keep
    assert ctx.workspace_bytes() == 0
    # a frame that fits still renders on the same context afterwards
    st, keep = _raw_particles(B, 50_000, 2e-3)
    rc = L.spl_render_noalloc(ctx.h, C.byref(st), C.byref(cam), C.byref(prm),
                              C.c_void_p(out.data_ptr()), None, stream)
    assert rc == B.SPL_OK, L.spl_last_error(ctx.h)
    torch.cuda.synchronize()
    assert float(out.sum()) > 0
    ctx.close()
