"""ctypes binding of libsplotch_hip.so (include/splotch.h).

Argument marshalling only: every render step runs in the HIP library.  Torch
tensors provide device memory and the current HIP stream.  There is no CPU
path: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsplotch_hip.so")

SPL_OK, SPL_EINVAL, SPL_ENOMEM, SPL_EDEVICE, SPL_EBUSY, SPL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SPL_F32, SPL_BF16, SPL_F16 = 0, 1, 2
SPL_ADD_RAW, SPL_ADD_AEQE, SPL_SORTED = 0, 1, 2
SPL_MAX_SPECIES = 8

EXPORTS = ["spl_create", "spl_destroy", "spl_last_error", "spl_workspace_bytes",
           "spl_scalar_range", "spl_project", "spl_bin", "spl_render_records", "spl_render",
           "spl_render_batch", "spl_autotune", "spl_set_timing", "spl_get_timing",
           "spl_set_option", "spl_render_noalloc", "spl_noalloc_scratch_bytes",
           "spl_dataset_upload", "spl_dataset_free", "spl_dataset_particles", "spl_dataset_bytes",
           "spl_render_dataset", "spl_render_batch_dataset", "spl_render_stream",
           "spl_host_alloc", "spl_host_free", "spl_trim"]
SPL_OPT_TIMING, SPL_OPT_GRAPHS, SPL_OPT_BATCH_BYTES, SPL_OPT_BATCH_PAIRS = 0, 1, 2, 3
SPL_N_STAGES = 9
STAGES = ["project", "count", "scan", "host_gap_items", "scatter", "sort", "large_splat",
          "splat", "finalise"]


class spl_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("h", C.c_void_p), ("intensity", C.c_void_p), ("scalar", C.c_void_p),
                ("attr_dtype", C.c_int32), ("h_scale", C.c_float), ("i_scale", C.c_float),
                ("s_scale", C.c_float), ("species", C.c_void_p),
                ("absorption", C.c_void_p), ("rgb", C.c_void_p), ("c_scale", C.c_float)]


class spl_camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("lookat", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("z_near", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class spl_look(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("n_entries", C.c_int32), ("log10_scalar", C.c_int32),
                ("brightness", C.c_double), ("lo", C.c_double), ("hi", C.c_double),
                ("vector_colour", C.c_int32)]


class spl_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_species", C.c_int32),
                ("looks", spl_look * SPL_MAX_SPECIES), ("k_sigma", C.c_double),
                ("sigma_min", C.c_double), ("nu", C.c_double), ("tile", C.c_int32),
                ("bin_rule", C.c_int32), ("large_cut", C.c_double), ("normalise", C.c_int32),
                ("flux_check", C.c_int32), ("deterministic", C.c_int32)]


class spl_stats(C.Structure):
    _fields_ = [("n_active", C.c_int64), ("n_large", C.c_int64), ("n_pairs", C.c_int64),
                ("n_large_pairs", C.c_int64), ("n_items", C.c_int64),
                ("flux", C.c_double * 3), ("max", C.c_double * 3), ("tile", C.c_int32),
                ("large_cut", C.c_double), ("raw_flux", C.c_double * 3),
                ("expected_flux", C.c_double * 3)]

    def as_dict(self):
        return {"n_active": self.n_active, "n_large": self.n_large, "n_pairs": self.n_pairs,
                "n_large_pairs": self.n_large_pairs, "n_items": self.n_items,
                "flux": list(self.flux), "max": list(self.max), "tile": self.tile,
                "large_cut": self.large_cut, "raw_flux": list(self.raw_flux),
                "expected_flux": list(self.expected_flux)}


_lib = None


def lib():
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.spl_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.spl_destroy.argtypes = [vp]
        L.spl_destroy.restype = None
        L.spl_last_error.argtypes = [vp]
        L.spl_last_error.restype = C.c_char_p
        L.spl_workspace_bytes.argtypes = [vp]
        L.spl_workspace_bytes.restype = i64
        L.spl_scalar_range.argtypes = [vp, C.POINTER(spl_particles), i32, i32,
                                       C.POINTER(d), C.POINTER(d), vp]
        L.spl_project.argtypes = [vp, C.POINTER(spl_particles), C.POINTER(spl_camera),
                                  C.POINTER(spl_params), vp, vp, vp]
        L.spl_bin.argtypes = [vp, i64, vp, vp, i32, i32, i32, d, i32, i32, vp, vp, vp, i64,
                              C.POINTER(i64), vp]
        L.spl_render_records.argtypes = [vp, i64, vp, vp, C.POINTER(spl_camera),
                                         C.POINTER(spl_params), vp, C.POINTER(spl_stats), vp]
        L.spl_render.argtypes = [vp, C.POINTER(spl_particles), C.POINTER(spl_camera),
                                 C.POINTER(spl_params), vp, C.POINTER(spl_stats), vp]
        L.spl_render_batch.argtypes = [vp, C.POINTER(spl_particles), i32, C.POINTER(spl_camera),
                                       C.POINTER(spl_params), C.POINTER(vp),
                                       C.POINTER(spl_stats), vp]
        L.spl_autotune.argtypes = [vp, C.POINTER(spl_particles), C.POINTER(spl_camera),
                                   C.POINTER(spl_params), C.POINTER(i32), C.POINTER(d), vp]
        L.spl_set_timing.argtypes = [vp, i32]
        L.spl_get_timing.argtypes = [vp, C.POINTER(d), C.POINTER(d), C.POINTER(i64)]
        L.spl_set_option.argtypes = [vp, i32, i64]
        L.spl_render_noalloc.argtypes = [vp, C.POINTER(spl_particles), C.POINTER(spl_camera),
                                         C.POINTER(spl_params), vp, C.POINTER(spl_stats), vp]
        L.spl_noalloc_scratch_bytes.argtypes = []
        L.spl_noalloc_scratch_bytes.restype = i64
        L.spl_dataset_upload.argtypes = [vp, C.POINTER(spl_particles), i32, i32, C.POINTER(vp),
                                         vp]
        L.spl_dataset_free.argtypes = [vp]
        L.spl_dataset_free.restype = None
        L.spl_dataset_particles.argtypes = [vp, C.POINTER(spl_particles)]
        L.spl_dataset_bytes.argtypes = [vp]
        L.spl_dataset_bytes.restype = i64
        L.spl_render_dataset.argtypes = [vp, vp, C.POINTER(spl_camera), C.POINTER(spl_params),
                                         vp, i32, C.POINTER(spl_stats), vp]
        L.spl_render_batch_dataset.argtypes = [vp, vp, i32, C.POINTER(spl_camera),
                                               C.POINTER(spl_params), C.POINTER(vp), i32,
                                               C.POINTER(spl_stats), vp]
        L.spl_render_stream.argtypes = [vp, C.POINTER(spl_particles), i64, C.POINTER(spl_camera),
                                        C.POINTER(spl_params), vp, i32, C.POINTER(spl_stats),
                                        vp]
        L.spl_host_alloc.argtypes = [C.c_size_t, C.POINTER(vp)]
        L.spl_host_free.argtypes = [vp]
        L.spl_host_free.restype = None
        L.spl_trim.argtypes = [vp]
        for name in EXPORTS:
            if name not in ("spl_destroy", "spl_last_error", "spl_workspace_bytes",
                            "spl_noalloc_scratch_bytes", "spl_dataset_free",
                            "spl_dataset_bytes", "spl_host_free"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class SplotchError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"splotch status {status}: {msg}")
        self.status = status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_camera(pose) -> spl_camera:
    c = spl_camera()
    c.eye[:] = list(map(float, pose.eye))
    c.lookat[:] = list(map(float, pose.lookat))
    c.up[:] = list(map(float, pose.up))
    c.fov_y_deg = float(pose.fov_y_deg)
    c.z_near = float(pose.z_near)
    c.width = int(pose.width)
    c.height = int(pose.height)
    return c


def host_particles(ps):
    """spl_particles over the host arrays of a particle set (FP32 attributes,
    unit scales); returns the struct and the arrays that keep it valid."""
    keep = []

    def arr(a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a.ctypes.data

    st = spl_particles()
    st.n = int(ps.x.shape[0])
    st.x, st.y, st.z = arr(ps.x, np.float32), arr(ps.y, np.float32), arr(ps.z, np.float32)
    st.h = arr(ps.h, np.float32)
    st.intensity = arr(ps.intensity, np.float32)
    st.scalar = arr(ps.scalar, np.float32)
    st.attr_dtype = SPL_F32
    st.h_scale = st.i_scale = st.s_scale = st.c_scale = 1.0
    st.species = arr(ps.species, np.uint8)
    st.absorption = arr(ps.absorption, np.float32)
    st.rgb = arr(getattr(ps, "rgb", None), np.float32)
    return st, keep


DTYPE_CODES = {"f32": SPL_F32, "bf16": SPL_BF16, "f16": SPL_F16}


class Dataset:
    """A particle set resident in device memory that the library owns
    (spl_dataset_upload): the host arrays are copied in and h, intensity,
    scalar and the colour vectors are converted to the stored dtype on the
    device.  `st` is the resident view (spl_dataset_particles)."""

    def __init__(self, ctx, ps, store="f32"):
        self.L = lib()
        self.code = DTYPE_CODES[store]
        src, keep = host_particles(ps)
        h = C.c_void_p()
        ctx._check(self.L.spl_dataset_upload(ctx.h, C.byref(src), 0, self.code, C.byref(h),
                                             _stream()))
        del keep
        self.h = h
        self.st = spl_particles()
        self.L.spl_dataset_particles(h, C.byref(self.st))
        self.n = int(src.n)
        self.device = f"cuda:{ctx.device}"

    def nbytes(self) -> int:
        return int(self.L.spl_dataset_bytes(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.L.spl_dataset_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_uploaders = {}


def _uploader(device):
    """One library context per device for uploads that have no context of
    their own."""
    import torch

    idx = torch.device(device).index or 0
    if idx not in _uploaders:
        _uploaders[idx] = Context(idx)
    return _uploaders[idx]


class DeviceParticles(Dataset):
    """A resident data set uploaded through a shared per-device context
    (the same conversion as Dataset)."""

    def __init__(self, ps, device="cuda:0", attr_dtype="f32"):
        super().__init__(_uploader(device), ps, attr_dtype)


class PinnedParticles:
    """Host copies of a particle set in page-locked memory (spl_host_alloc),
    the input of out-of-core rendering (spl_render_stream).  attrs: optional
    stored smoothing length, intensity and scalar arrays (dict with keys h,
    intensity, scalar, in the layout of attr_dtype, e.g. BF16 bit patterns as
    uint16) to use instead of the set's FP32 values; the scales stay 1."""

    def __init__(self, ps, attrs=None, attr_dtype=SPL_F32):
        self.L = lib()
        self.blocks = []

        def pin(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dt)
            p = C.c_void_p()
            if self.L.spl_host_alloc(a.nbytes, C.byref(p)) != SPL_OK:
                raise SplotchError(SPL_ENOMEM, "spl_host_alloc failed")
            self.blocks.append(p)
            C.memmove(p, a.ctypes.data, a.nbytes)
            return p.value

        st = spl_particles()
        st.n = int(ps.x.shape[0])
        st.x, st.y, st.z = pin(ps.x, np.float32), pin(ps.y, np.float32), pin(ps.z, np.float32)
        if attrs is None:
            st.h = pin(ps.h, np.float32)
            st.intensity = pin(ps.intensity, np.float32)
            st.scalar = pin(ps.scalar, np.float32)
            st.attr_dtype = SPL_F32
        else:
            st.h = pin(attrs["h"], attrs["h"].dtype)
            st.intensity = pin(attrs["intensity"], attrs["intensity"].dtype)
            st.scalar = pin(attrs["scalar"], attrs["scalar"].dtype)
            st.attr_dtype = attr_dtype
        st.h_scale = st.i_scale = st.s_scale = st.c_scale = 1.0
        st.species = pin(ps.species, np.uint8)
        st.absorption = None
        st.rgb = pin(getattr(ps, "rgb", None), np.float32) if attrs is None else None
        self.st = st
        self.n = st.n

    def close(self):
        for p in self.blocks:
            self.L.spl_host_free(p)
        self.blocks = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Palettes:
    """Device copies of the colour maps (one per species)."""

    def __init__(self, pals, device="cuda:0"):
        import torch

        self.t = [torch.from_numpy(np.ascontiguousarray(p, np.float32).reshape(-1, 3)).to(device)
                  for p in pals]


def make_params(mode, palettes: Palettes, looks, k_sigma=1.0 / 3.0, sigma_min=0.5, nu=3.0,
                tile=0, bin_rule=0, large_cut=0.0, normalise=0, flux_check=0,
                deterministic=0) -> spl_params:
    """looks: list of dicts with brightness, lo, hi, log10 and vector (1: the
    species takes its colour from the particles' rgb vectors), one per
    species.  The returned parameters keep `palettes` alive: they hold its
    device pointers."""
    p = spl_params()
    p._palettes = palettes
    p.mode = mode
    p.n_species = len(looks)
    for k, l in enumerate(looks):
        p.looks[k].rgb = palettes.t[k].data_ptr()
        p.looks[k].n_entries = palettes.t[k].shape[0]
        p.looks[k].log10_scalar = int(l.get("log10", 0))
        p.looks[k].brightness = float(l.get("brightness", 1.0))
        p.looks[k].lo = float(l.get("lo", 0.0))
        p.looks[k].hi = float(l.get("hi", 1.0))
        p.looks[k].vector_colour = int(l.get("vector", 0))
    p.k_sigma = k_sigma
    p.sigma_min = sigma_min
    p.nu = nu
    p.tile = tile
    p.bin_rule = bin_rule
    p.large_cut = large_cut
    p.normalise = normalise
    p.flux_check = flux_check
    p.deterministic = deterministic
    return p


class Context:
    """One library context on one device (spl_create / spl_destroy)."""

    def __init__(self, device: int = 0):
        self.L = lib()
        h = C.c_void_p()
        rc = self.L.spl_create(device, C.byref(h))
        if rc != SPL_OK:
            raise SplotchError(rc, f"spl_create({device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.L.spl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != SPL_OK:
            raise SplotchError(rc, self.L.spl_last_error(self.h).decode())

    def workspace_bytes(self) -> int:
        return int(self.L.spl_workspace_bytes(self.h))

    def spl_trim(self):
        self._check(self.L.spl_trim(self.h))

    def spl_scalar_range(self, parts: DeviceParticles, n_species: int, log10: bool):
        lo = (C.c_double * n_species)()
        hi = (C.c_double * n_species)()
        self._check(self.L.spl_scalar_range(self.h, C.byref(parts.st), n_species, int(log10),
                                            lo, hi, _stream()))
        return list(lo), list(hi)

    def spl_project(self, parts: DeviceParticles, pose, prm: spl_params, with_rec2=False):
        import torch

        rec = torch.empty((parts.n, 8), dtype=torch.float32, device=parts.device)
        rec2 = torch.empty((parts.n, 2), dtype=torch.float32, device=parts.device) if with_rec2 else None
        cam = make_camera(pose)
        self._check(self.L.spl_project(self.h, C.byref(parts.st), C.byref(cam), C.byref(prm),
                                       _ptr(rec), _ptr(rec2), _stream()))
        return rec, rec2

    def spl_bin(self, rec, rec2, width, height, tile, nu=3.0, bin_rule=0, by_depth=False):
        import torch

        n = rec.shape[0]
        ntx = (width + tile - 1) // tile
        nty = (height + tile - 1) // tile
        dev = rec.device
        counts = torch.empty(ntx * nty, dtype=torch.int32, device=dev)
        offsets = torch.empty(ntx * nty + 1, dtype=torch.int32, device=dev)
        npairs = C.c_int64()
        self._check(self.L.spl_bin(self.h, n, _ptr(rec), _ptr(rec2), width, height, tile, nu,
                                   bin_rule, int(by_depth), _ptr(counts), _ptr(offsets), None, 0,
                                   C.byref(npairs), _stream()))
        pairs = torch.empty(max(npairs.value, 1), dtype=torch.int32, device=dev)
        self._check(self.L.spl_bin(self.h, n, _ptr(rec), _ptr(rec2), width, height, tile, nu,
                                   bin_rule, int(by_depth), _ptr(counts), _ptr(offsets),
                                   _ptr(pairs), pairs.shape[0], C.byref(npairs), _stream()))
        return counts, offsets, pairs[: npairs.value]

    def spl_render_records(self, rec, rec2, pose, prm: spl_params, out=None, stats=True):
        import torch

        if out is None:
            out = torch.empty((pose.height, pose.width, 3), dtype=torch.float32, device=rec.device)
        st = spl_stats()
        cam = make_camera(pose)
        self._check(self.L.spl_render_records(self.h, rec.shape[0], _ptr(rec), _ptr(rec2),
                                              C.byref(cam), C.byref(prm), _ptr(out),
                                              C.byref(st) if stats else None, _stream()))
        return out, (st.as_dict() if stats else None)

    def spl_render(self, parts: DeviceParticles, pose, prm: spl_params, out=None, stats=True):
        import torch

        if out is None:
            out = torch.empty((pose.height, pose.width, 3), dtype=torch.float32, device=parts.device)
        st = spl_stats()
        cam = make_camera(pose)
        self._check(self.L.spl_render(self.h, C.byref(parts.st), C.byref(cam), C.byref(prm),
                                      _ptr(out), C.byref(st) if stats else None, _stream()))
        return out, (st.as_dict() if stats else None)

    def spl_render_noalloc(self, parts: DeviceParticles, pose, prm: spl_params, out=None,
                           stats=True):
        import torch

        if out is None:
            out = torch.empty((pose.height, pose.width, 3), dtype=torch.float32, device=parts.device)
        st = spl_stats()
        cam = make_camera(pose)
        self._check(self.L.spl_render_noalloc(self.h, C.byref(parts.st), C.byref(cam),
                                              C.byref(prm), _ptr(out),
                                              C.byref(st) if stats else None, _stream()))
        return out, (st.as_dict() if stats else None)

    def spl_render_batch(self, parts: DeviceParticles, poses, prms, outs=None, stats=True):
        import torch

        nv = len(poses)
        if outs is None:
            outs = [torch.empty((p.height, p.width, 3), dtype=torch.float32, device=parts.device)
                    for p in poses]
        cams = (spl_camera * nv)(*[make_camera(p) for p in poses])
        prm_arr = (spl_params * nv)(*prms)
        out_arr = (C.c_void_p * nv)(*[o.data_ptr() for o in outs])
        sts = (spl_stats * nv)()
        self._check(self.L.spl_render_batch(self.h, C.byref(parts.st), nv, cams, prm_arr, out_arr,
                                            sts if stats else None, _stream()))
        return outs, ([s.as_dict() for s in sts] if stats else None)

    def spl_render_dataset(self, ds: Dataset, pose, prm: spl_params, out=None, host_out=False,
                           stats=True):
        """host_out: the image comes back as a numpy array filled by the
        library (device image copied to host memory)."""
        import torch

        if out is None:
            out = (np.empty((pose.height, pose.width, 3), np.float32) if host_out else
                   torch.empty((pose.height, pose.width, 3), dtype=torch.float32,
                               device=ds.device))
        ptr = out.ctypes.data if host_out else out.data_ptr()
        st = spl_stats()
        cam = make_camera(pose)
        self._check(self.L.spl_render_dataset(self.h, ds.h, C.byref(cam), C.byref(prm),
                                              C.c_void_p(ptr), 0 if host_out else 1,
                                              C.byref(st) if stats else None, _stream()))
        return out, (st.as_dict() if stats else None)

    def spl_render_batch_dataset(self, ds: Dataset, poses, prms, outs=None, host_out=False,
                                 stats=True):
        import torch

        nv = len(poses)
        if outs is None:
            outs = [np.empty((p.height, p.width, 3), np.float32) if host_out else
                    torch.empty((p.height, p.width, 3), dtype=torch.float32, device=ds.device)
                    for p in poses]
        cams = (spl_camera * nv)(*[make_camera(p) for p in poses])
        prm_arr = (spl_params * nv)(*prms)
        out_arr = (C.c_void_p * nv)(*[o.ctypes.data if host_out else o.data_ptr() for o in outs])
        sts = (spl_stats * nv)()
        self._check(self.L.spl_render_batch_dataset(self.h, ds.h, nv, cams, prm_arr, out_arr,
                                                    0 if host_out else 1,
                                                    sts if stats else None, _stream()))
        return outs, ([s.as_dict() for s in sts] if stats else None)

    def spl_render_stream(self, host: PinnedParticles, chunk: int, pose, prm: spl_params,
                          out=None, host_out=False, stats=True, device="cuda:0"):
        import torch

        if out is None:
            out = (np.empty((pose.height, pose.width, 3), np.float32) if host_out else
                   torch.empty((pose.height, pose.width, 3), dtype=torch.float32, device=device))
        ptr = out.ctypes.data if host_out else out.data_ptr()
        st = spl_stats()
        cam = make_camera(pose)
        self._check(self.L.spl_render_stream(self.h, C.byref(host.st), int(chunk), C.byref(cam),
                                             C.byref(prm), C.c_void_p(ptr), 0 if host_out else 1,
                                             C.byref(st) if stats else None, _stream()))
        return out, (st.as_dict() if stats else None)

    def spl_set_option(self, option: int, value: int):
        self._check(self.L.spl_set_option(self.h, option, int(value)))

    def spl_set_timing(self, enable: bool):
        self._check(self.L.spl_set_timing(self.h, int(enable)))

    def spl_get_timing(self):
        ms = (C.c_double * SPL_N_STAGES)()
        by = (C.c_double * SPL_N_STAGES)()
        fr = C.c_int64()
        self._check(self.L.spl_get_timing(self.h, ms, by, C.byref(fr)))
        return list(ms), list(by), fr.value

    def spl_autotune(self, parts: DeviceParticles, pose, prm: spl_params):
        tile = C.c_int32()
        cut = C.c_double()
        cam = make_camera(pose)
        self._check(self.L.spl_autotune(self.h, C.byref(parts.st), C.byref(cam), C.byref(prm),
                                        C.byref(tile), C.byref(cut), _stream()))
        return tile.value, cut.value
