"""Colour from a vector field, the FP64 expected-flux check and out-of-core
rendering, on the GPU through the C ABI, against the FP64 oracle.

* Vector colour (Sect. 2.1: colour taken directly from a vector input field):
  all three transfer modes, FP32 and BF16 storage, species mixing palette and
  vector colouring.
* Expected flux: sum_p E_p kappa_p from the library against the oracle's,
  and against the flux of the additive sum J the splat produced.
* Out-of-core rendering (Sect. 3.1: chunks copied through two device buffers
  while the previous one renders; the image accumulates over chunks): the
  streamed image against the resident render and the oracle, with ragged
  chunks, pinned and pageable host memory, host output."""
import ctypes as C

import numpy as np
import pytest

from paper_1606_04427_amd import synth
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-3}


@pytest.fixture(scope="module")
def env(oracle):
    import torch

    from paper_1606_04427_amd import binding as B

    assert torch.cuda.is_available()
    ctx = B.Context(0)
    yield B, ctx, oracle
    ctx.close()


def _set(n, seed, absorption=True):
    ps = synth.soneira_peebles(n, seed=seed, absorption=absorption)
    ps.rgb = synth.colour_field(ps, seed=seed + 1)
    looks, pals = [], []
    for k in range(2):
        s = ps.scalar[ps.species == k]
        looks.append(dict(log10=1, brightness=0.03 * (1 + k), lo=float(np.log10(s.min())),
                          hi=float(np.log10(s.max()))))
        pals.append(synth.palette(k))
    return ps, looks, pals


@pytest.mark.parametrize("store", ["f32", "bf16"])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("mix", [False, True])
def test_vector_colour_matches_oracle(env, store, mode, mix):
    import torch

    B, ctx, R = env
    ps, looks, pals = _set(200_000, 81)
    looks = [dict(l) for l in looks]
    looks[1]["vector"] = 1
    if not mix:
        looks[0]["vector"] = 1
    print(f"vector colour store={store} mode={mode} mix={mix}", flush=True)
    ds = B.Dataset(ctx, ps, store)
    P = B.Palettes(pals)
    prm = B.make_params(mode, P, looks, tile=16)
    pose = synth.random_poses(1, seed=420 + mode, width=384, height=320)[0]
    img, st = ctx.spl_render_dataset(ds, pose, prm)
    torch.cuda.synchronize()
    got = img.cpu().numpy().astype(np.float64)
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    want = R.render(R.Particles(ps), pose, R.params(mode, L))
    assert st["n_active"] > 1000
    assert rel_l2(got, want) < TOL[store]
    ds.close()


def test_vector_colour_needs_the_rgb_array(env):
    B, ctx, _ = env
    ps, looks, pals = _set(2000, 83)
    ps.rgb = None
    looks[0]["vector"] = 1
    ds = B.Dataset(ctx, ps, "f32")
    prm = B.make_params(1, B.Palettes(pals), looks, tile=16)
    with pytest.raises(B.SplotchError) as e:
        ctx.spl_render_dataset(ds, synth.random_poses(1, seed=3)[0], prm)
    assert e.value.status == B.SPL_EINVAL and "rgb" in str(e.value)
    ds.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("cut", [-1.0, 16.0])
def test_expected_flux_matches_oracle_and_image(env, mode, cut):
    import torch

    B, ctx, R = env
    ps, looks, pals = _set(300_000, 85, absorption=False)
    ds = B.Dataset(ctx, ps, "f32")
    P = B.Palettes(pals)
    prm = B.make_params(mode, P, looks, tile=16, large_cut=cut, flux_check=1)
    pose = synth.random_poses(1, seed=431, width=512, height=384, dist_range=(0.6, 0.9))[0]
    print(f"expected flux mode={mode} cut={cut}", flush=True)
    img, st = ctx.spl_render_dataset(ds, pose, prm)
    torch.cuda.synchronize()
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    RP = R.Particles(ps)
    want_exp = R.expected_flux(RP, pose, R.params(mode, L))
    raw = R.render(RP, pose, R.params(R.ADD_RAW, L))
    np.testing.assert_allclose(st["expected_flux"], want_exp, rtol=1e-5)
    # conservation: what the splat put into J equals the expected flux
    np.testing.assert_allclose(st["raw_flux"], st["expected_flux"], rtol=1e-5)
    np.testing.assert_allclose(st["raw_flux"], raw.reshape(-1, 3).sum(0), rtol=1e-5)
    # the flux of the output image (after the map in absorption = emission mode)
    np.testing.assert_allclose(st["flux"], img.cpu().numpy().astype(np.float64).reshape(-1, 3).sum(0),
                               rtol=1e-9)
    # without the check the field is NaN, and sorted mode never has one
    _, st0 = ctx.spl_render_dataset(ds, pose, B.make_params(mode, P, looks, tile=16))
    assert all(np.isnan(st0["expected_flux"]))
    ds.close()


def test_expected_flux_in_a_batch(env):
    B, ctx, R = env
    ps, looks, pals = _set(150_000, 87, absorption=False)
    ds = B.Dataset(ctx, ps, "f32")
    P = B.Palettes(pals)
    poses = [synth.random_poses(1, seed=440 + k, width=w, height=h)[0]
             for k, (w, h) in enumerate([(256, 256), (320, 200)])]
    prms = [B.make_params(m, P, looks, tile=16, flux_check=1) for m in (1, 0)]
    _, sts = ctx.spl_render_batch_dataset(ds, poses, prms)
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    RP = R.Particles(ps)
    for pose, prm, st in zip(poses, (1, 0), sts):
        want = R.expected_flux(RP, pose, R.params(prm, L))
        np.testing.assert_allclose(st["expected_flux"], want, rtol=1e-5)
        np.testing.assert_allclose(st["raw_flux"], st["expected_flux"], rtol=1e-5)
    ds.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("pinned", [True, False])
def test_streamed_render_equals_resident_and_oracle(env, mode, pinned):
    import torch

    B, ctx, R = env
    ps, looks, pals = _set(400_000, 89, absorption=False)
    P = B.Palettes(pals)
    prm = B.make_params(mode, P, looks, tile=16, large_cut=32.0, flux_check=1)
    pose = synth.random_poses(1, seed=450, width=512, height=384, dist_range=(0.6, 1.2))[0]
    chunk = 70_000  # 6 chunks, the last one ragged
    print(f"stream mode={mode} pinned={pinned} chunk={chunk}", flush=True)
    ds = B.Dataset(ctx, ps, "f32")
    res, st_res = ctx.spl_render_dataset(ds, pose, prm)
    if pinned:
        host = B.PinnedParticles(ps)
    else:
        st_h, keep = B.host_particles(ps)
        host = type("Host", (), {"st": st_h, "n": ps.n})()
    img, st = ctx.spl_render_stream(host, chunk, pose, prm)
    torch.cuda.synchronize()
    got = img.cpu().numpy().astype(np.float64)
    assert st["n_active"] == st_res["n_active"]
    assert st["n_pairs"] == st_res["n_pairs"]
    assert rel_l2(got, res.cpu().numpy()) < 1e-6
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    want = R.render(R.Particles(ps), pose, R.params(mode, L))
    assert rel_l2(got, want) < 1e-5
    np.testing.assert_allclose(st["raw_flux"], st_res["raw_flux"], rtol=1e-6)
    np.testing.assert_allclose(st["expected_flux"], st_res["expected_flux"], rtol=1e-9)
    # host output of the same streamed frame
    himg, _ = ctx.spl_render_stream(host, chunk, pose, prm, host_out=True)
    assert rel_l2(himg, got) < 1e-6
    # one chunk larger than the set
    one, st1 = ctx.spl_render_stream(host, 10 * ps.n, pose, prm)
    assert rel_l2(one.cpu().numpy(), got) < 1e-6
    if pinned:
        host.close()
    ds.close()


def test_stream_refuses_sorted_mode_and_bad_chunks(env):
    B, ctx, _ = env
    ps, looks, pals = _set(5000, 91)
    host = B.PinnedParticles(ps)
    P = B.Palettes(pals)
    pose = synth.random_poses(1, seed=5, width=64, height=64)[0]
    with pytest.raises(B.SplotchError) as e:
        ctx.spl_render_stream(host, 1000, pose, B.make_params(2, P, looks))
    assert e.value.status == B.SPL_EUNSUPPORTED
    with pytest.raises(B.SplotchError) as e:
        ctx.spl_render_stream(host, 0, pose, B.make_params(1, P, looks))
    assert e.value.status == B.SPL_EINVAL
    host.close()


def test_stream_of_an_empty_set(env):
    import torch

    B, ctx, _ = env
    ps, looks, pals = _set(1000, 93, absorption=False)
    empty = ps.subset(np.arange(0))
    st_h, keep = B.host_particles(empty)
    host = type("Host", (), {"st": st_h, "n": 0})()
    img, st = ctx.spl_render_stream(host, 100, synth.random_poses(1, seed=6, width=32,
                                                                  height=16)[0],
                                    B.make_params(1, B.Palettes(pals), looks))
    torch.cuda.synchronize()
    assert float(img.abs().sum()) == 0.0 and st["n_active"] == 0


def test_streamed_frame_from_bf16_host_attributes(env):
    """Out-of-core frame whose host arrays hold BF16 attributes (rounded to
    nearest even on the host): the same stored bits as a BF16 data set, so
    the streamed image equals that data set's resident render to rounding,
    and the oracle on the FP32 originals within the BF16 bar."""
    import torch

    B, ctx, R = env
    ps, looks, pals = _set(300_000, 95, absorption=False)
    P = B.Palettes(pals)
    prm = B.make_params(1, P, looks, tile=16, large_cut=32.0)
    pose = synth.random_poses(1, seed=452, width=384, height=256, dist_range=(0.6, 1.2))[0]
    print("stream bf16 host attributes", flush=True)
    ds = B.Dataset(ctx, ps, "bf16")
    res, st_res = ctx.spl_render_dataset(ds, pose, prm)

    def bits(a):
        u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
        return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)

    host = B.PinnedParticles(ps, {"h": bits(ps.h), "intensity": bits(ps.intensity),
                                  "scalar": bits(ps.scalar)}, B.SPL_BF16)
    img, st = ctx.spl_render_stream(host, 70_000, pose, prm)  # 5 chunks, ragged
    torch.cuda.synchronize()
    host.close()
    got = img.cpu().numpy().astype(np.float64)
    assert st["n_active"] == st_res["n_active"] and st["n_pairs"] == st_res["n_pairs"]
    assert rel_l2(got, res.cpu().numpy()) < 1e-6
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    want = R.render(R.Particles(ps), pose, R.params(1, L))
    assert rel_l2(got, want) < TOL["bf16"]
    ds.close()
