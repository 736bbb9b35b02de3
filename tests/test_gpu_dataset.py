"""Resident data sets and host output through the C ABI.

spl_dataset_upload converts h, intensity, scalar and colour vectors on the
device; the stored bits must equal a host-side conversion of the same values
(FP32 as is, BF16 and FP16 rounded to nearest even, FP16 with the power-of-two
scale that puts the largest magnitude in [2^10, 2^11)).  A render through the
handle must equal the render of the same arrays passed as raw device pointers
(bit for bit in the depth-sorted mode, whose compositing is deterministic;
additive images differ only in the order of float additions), and the host
output must equal the device output of the same call."""
import ctypes as C
import math

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


def _looks(ps):
    looks, pals = [], []
    for k in range(2):
        s = ps.scalar[ps.species == k]
        looks.append(dict(log10=1, brightness=0.03 * (1 + k), lo=float(np.log10(s.min())),
                          hi=float(np.log10(s.max()))))
        pals.append(synth.palette(k))
    return looks, pals


def _bf16_bits(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def _f16_scale(a):
    a = np.asarray(a, np.float64)
    m = float(np.abs(a[np.isfinite(a)]).max())
    return 2.0 ** math.floor(math.log2(m / 1024.0)) if m > 0 else 1.0


def _hip():
    """The HIP runtime this process already uses (torch and the library share
    it); opened by its loaded path so that no second copy is loaded."""
    with open("/proc/self/maps") as f:
        paths = {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    assert len(paths) == 1, paths
    hip = C.CDLL(paths.pop())
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return hip


def _download(ptr, count, dtype):
    """count values of the given dtype at device address ptr, to the host."""
    import torch

    torch.cuda.synchronize()
    buf = np.empty(count, dtype)
    hip_memcpy_device_to_host = 2
    rc = _hip().hipMemcpy(C.c_void_p(buf.ctypes.data), C.c_void_p(ptr), buf.nbytes,
                          hip_memcpy_device_to_host)
    assert rc == 0
    return buf


@pytest.mark.parametrize("store", ["f32", "bf16", "f16"])
def test_upload_converts_like_the_host(env, store):
    B, ctx, _ = env
    ps = synth.soneira_peebles(50_000, seed=71, absorption=True)
    ps.rgb = synth.colour_field(ps, seed=72)
    print(f"dataset upload store={store} n={ps.n}", flush=True)
    ds = B.Dataset(ctx, ps, store)
    st = ds.st
    assert st.n == ps.n and st.attr_dtype == B.DTYPE_CODES[store]
    for f, ptr in (("x", st.x), ("y", st.y), ("z", st.z), ("absorption", st.absorption)):
        got = _download(ptr, ps.n, np.float32)
        assert np.array_equal(got.view(np.uint32), getattr(ps, f).view(np.uint32)), f
    assert np.array_equal(_download(st.species, ps.n, np.uint8), ps.species)
    arrays = [("h", ps.h, st.h, st.h_scale), ("intensity", ps.intensity, st.intensity, st.i_scale),
              ("scalar", ps.scalar, st.scalar, st.s_scale),
              ("rgb", ps.rgb.reshape(-1), st.rgb, st.c_scale)]
    for name, a, ptr, scale in arrays:
        if store == "f32":
            assert scale == 1.0
            got = _download(ptr, a.size, np.float32)
            assert np.array_equal(got.view(np.uint32), a.view(np.uint32)), name
        elif store == "bf16":
            assert scale == 1.0
            got = _download(ptr, a.size, np.uint16)
            assert np.array_equal(got, _bf16_bits(a)), name
        else:
            want_scale = _f16_scale(a)
            assert scale == want_scale, name
            want = (np.asarray(a, np.float64) / want_scale).astype(np.float32).astype(np.float16)
            got = _download(ptr, a.size, np.uint16)
            assert np.array_equal(got, want.view(np.uint16)), name
    assert ds.nbytes() >= ps.n * (12 + 1 + 4)
    ds.close()


def _raw(B, ps):
    """The same particle set as raw device pointers (FP32), without the
    library's upload."""
    import torch

    t = {f: torch.from_numpy(np.ascontiguousarray(getattr(ps, f))).cuda()
         for f in ("x", "y", "z", "h", "intensity", "scalar", "species", "absorption")}
    st = B.spl_particles()
    st.n = ps.n
    st.x, st.y, st.z = t["x"].data_ptr(), t["y"].data_ptr(), t["z"].data_ptr()
    st.h, st.intensity, st.scalar = (t["h"].data_ptr(), t["intensity"].data_ptr(),
                                     t["scalar"].data_ptr())
    st.attr_dtype = B.SPL_F32
    st.h_scale = st.i_scale = st.s_scale = st.c_scale = 1.0
    st.species = t["species"].data_ptr()
    st.absorption = t["absorption"].data_ptr()
    st.rgb = None
    return st, t


@pytest.mark.parametrize("mode", [1, 2])
def test_render_through_the_handle_equals_raw_pointers(env, mode):
    import torch

    B, ctx, R = env
    ps = synth.soneira_peebles(200_000, seed=73, absorption=True)
    looks, pals = _looks(ps)
    P = B.Palettes(pals)
    prm = B.make_params(mode, P, looks, tile=16, large_cut=32.0 if mode != 2 else 0.0)
    pose = synth.random_poses(1, seed=404, width=320, height=240)[0]
    print(f"handle vs raw mode={mode}", flush=True)
    ds = B.Dataset(ctx, ps, "f32")
    img_ds, st_ds = ctx.spl_render_dataset(ds, pose, prm)
    raw, keep = _raw(B, ps)
    out = torch.empty((240, 320, 3), device="cuda:0")
    st = B.spl_stats()
    cam = B.make_camera(pose)
    rc = ctx.L.spl_render(ctx.h, C.byref(raw), C.byref(cam), C.byref(prm),
                          C.c_void_p(out.data_ptr()), C.byref(st),
                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.SPL_OK
    torch.cuda.synchronize()
    a = img_ds.cpu().numpy()
    b = out.cpu().numpy()
    assert st_ds["n_active"] == st.n_active and st_ds["n_pairs"] == st.n_pairs
    if mode == 2:
        assert np.array_equal(a, b)
    else:
        assert rel_l2(a, b) < 1e-6
    # host output: the same call filling host memory
    host, st_h = ctx.spl_render_dataset(ds, pose, prm, host_out=True)
    assert isinstance(host, np.ndarray)
    if mode == 2:
        assert np.array_equal(host, a)
    else:
        assert rel_l2(host, a) < 1e-6
    L = R.Looks([dict(rgb=p, **l) for p, l in zip(pals, looks)])
    want = R.render(R.Particles(ps), pose, R.params(mode, L))
    assert rel_l2(host, want) < 1e-5
    ds.close()


def test_batch_through_the_handle_with_host_output(env):
    import torch

    B, ctx, R = env
    ps = synth.soneira_peebles(150_000, seed=74)
    looks, pals = _looks(ps)
    P = B.Palettes(pals)
    poses = [synth.random_poses(1, seed=410 + k, width=w, height=h)[0]
             for k, (w, h) in enumerate([(256, 256), (200, 120), (384, 256)])]
    prms = [B.make_params(m, P, looks, tile=16) for m in (1, 0, 1)]
    ds = B.Dataset(ctx, ps, "f32")
    dev, sts = ctx.spl_render_batch_dataset(ds, poses, prms)
    host, sts_h = ctx.spl_render_batch_dataset(ds, poses, prms, host_out=True)
    torch.cuda.synchronize()
    for d, h, s1, s2 in zip(dev, host, sts, sts_h):
        assert isinstance(h, np.ndarray) and h.shape == tuple(d.shape)
        assert rel_l2(h, d.cpu().numpy()) < 1e-6
        assert s1["n_pairs"] == s2["n_pairs"]
    ds.close()


def test_dataset_errors(env):
    B, ctx, _ = env
    ps = synth.blobs(1000, seed=75)
    src, keep = B.host_particles(ps)
    h = C.c_void_p()
    stream = None
    assert ctx.L.spl_dataset_upload(ctx.h, C.byref(src), 0, 7, C.byref(h), stream) == B.SPL_EINVAL
    bad = B.spl_particles.from_buffer_copy(src)
    bad.x = None
    assert ctx.L.spl_dataset_upload(ctx.h, C.byref(bad), 0, 0, C.byref(h), stream) == B.SPL_EINVAL
    assert not h.value
    # NULL data set handle
    cam = B.make_camera(synth.blobs_camera(32, 32))
    prm = B.make_params(1, B.Palettes([synth.palette(0)]), [dict(log10=0)])
    rc = ctx.L.spl_render_dataset(ctx.h, None, C.byref(cam), C.byref(prm), None, 1, None, None)
    assert rc == B.SPL_EINVAL
    assert b"data set" in ctx.L.spl_last_error(ctx.h)
