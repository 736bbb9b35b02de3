"""ctypes binding of the FP64 CPU oracle (libsplref.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg.  The product package never imports it.

`build()` compiles oracle/splref.c with gcc (no contraction, no fast-math).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "splref.c")
LIB = os.path.join(HERE, "libsplref.so")

ADD_RAW, ADD_AEQE, SORTED = 0, 1, 2


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("lookat", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("z_near", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class _Look(C.Structure):
    _fields_ = [("rgb", C.POINTER(C.c_float)), ("n_entries", C.c_int32),
                ("log10_scalar", C.c_int32), ("brightness", C.c_double),
                ("lo", C.c_double), ("hi", C.c_double), ("vector_colour", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_species", C.c_int32), ("looks", C.POINTER(_Look)),
                ("k_sigma", C.c_double), ("sigma_min", C.c_double), ("nu", C.c_double),
                ("normalise", C.c_int32)]


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("z", C.POINTER(C.c_double)), ("h", C.POINTER(C.c_double)),
                ("intensity", C.POINTER(C.c_double)), ("scalar", C.POINTER(C.c_double)),
                ("absorption", C.POINTER(C.c_double)), ("species", C.POINTER(C.c_uint8)),
                ("rgb", C.POINTER(C.c_double))]


class Proj(C.Structure):
    _fields_ = [("X", C.c_double), ("Y", C.c_double), ("zv", C.c_double),
                ("rho", C.c_double), ("sigma", C.c_double), ("R", C.c_double),
                ("E", C.c_double * 3), ("a", C.c_double), ("active", C.c_int32),
                ("i0", C.c_int32), ("i1", C.c_int32), ("j0", C.c_int32), ("j1", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp, fp, u32p, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_float),
                              C.POINTER(C.c_uint32), C.POINTER(C.c_int32))
        L.sr_frame.argtypes = [C.POINTER(_Camera), dp]
        L.sr_validate.argtypes = [C.POINTER(_Camera), C.POINTER(_Params)]
        L.sr_project.argtypes = [C.POINTER(_Particles), C.POINTER(_Camera), C.POINTER(_Params),
                                 C.POINTER(Proj)]
        L.sr_scalar_range.argtypes = [C.POINTER(_Particles), C.c_int32, C.c_int32, dp, dp]
        L.sr_render.argtypes = [C.POINTER(_Particles), C.POINTER(_Camera), C.POINTER(_Params), dp]
        L.sr_render_brute.argtypes = [C.POINTER(_Particles), C.POINTER(_Camera),
                                      C.POINTER(_Params), C.c_int32, dp]
        L.sr_render_sorted_back_to_front.argtypes = [C.POINTER(_Particles), C.POINTER(_Camera),
                                                     C.POINTER(_Params), dp]
        L.sr_record_box.argtypes = [fp, C.c_float, C.c_int32, C.c_int32, i32p, i32p, i32p, i32p]
        L.sr_bin_records.argtypes = [C.c_int64, fp, fp, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_float, C.c_int32, C.c_int32, u32p, u32p, u32p,
                                     C.c_int64, C.POINTER(C.c_int64)]
        L.sr_render_records.argtypes = [C.c_int64, fp, fp, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_double, dp]
        L.sr_expected_flux.argtypes = [C.POINTER(_Particles), C.POINTER(_Camera),
                                       C.POINTER(_Params), dp]
        L.sr_image_stats.argtypes = [dp, C.c_int32, C.c_int32, dp, dp]
        L.sr_image_stats.restype = None
        _lib = L
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def camera(pose) -> _Camera:
    c = _Camera()
    c.eye[:] = list(pose.eye)
    c.lookat[:] = list(pose.lookat)
    c.up[:] = list(pose.up)
    c.fov_y_deg = float(pose.fov_y_deg)
    c.z_near = float(pose.z_near)
    c.width = int(pose.width)
    c.height = int(pose.height)
    return c


class Looks:
    """Keeps the palettes alive while the C structs point at them."""

    def __init__(self, looks):
        # a species coloured from the vector field needs no palette
        self.pals = [np.ascontiguousarray(l.get("rgb", np.zeros((1, 3))), dtype=np.float32)
                     for l in looks]
        self.arr = (_Look * len(looks))()
        for k, l in enumerate(looks):
            self.arr[k].rgb = _ptr(self.pals[k], C.c_float)
            self.arr[k].n_entries = self.pals[k].shape[0]
            self.arr[k].log10_scalar = int(l.get("log10", 0))
            self.arr[k].brightness = float(l.get("brightness", 1.0))
            self.arr[k].lo = float(l.get("lo", 0.0))
            self.arr[k].hi = float(l.get("hi", 1.0))
            self.arr[k].vector_colour = int(l.get("vector", 0))


def params(mode, looks: Looks, k_sigma=1.0 / 3.0, sigma_min=0.5, nu=3.0, normalise=0) -> _Params:
    p = _Params()
    p.mode = mode
    p.n_species = len(looks.pals)
    p.looks = C.cast(looks.arr, C.POINTER(_Look))
    p.k_sigma = k_sigma
    p.sigma_min = sigma_min
    p.nu = nu
    p.normalise = normalise
    return p


class Particles:
    """FP64 copies of a particle set (inputs widened exactly from float32)."""

    def __init__(self, ps, absorption=None, rgb=None):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.x, self.y, self.z = f64(ps.x), f64(ps.y), f64(ps.z)
        self.h, self.i, self.s = f64(ps.h), f64(ps.intensity), f64(ps.scalar)
        a = absorption if absorption is not None else ps.absorption
        self.a = None if a is None else f64(a)
        self.sp = np.ascontiguousarray(ps.species, dtype=np.uint8)
        c = rgb if rgb is not None else getattr(ps, "rgb", None)
        self.rgb = None if c is None else f64(np.asarray(c).reshape(-1, 3))
        self.st = _Particles()
        self.st.n = self.x.shape[0]
        self.st.x, self.st.y, self.st.z = (_ptr(self.x, C.c_double), _ptr(self.y, C.c_double),
                                           _ptr(self.z, C.c_double))
        self.st.h = _ptr(self.h, C.c_double)
        self.st.intensity = _ptr(self.i, C.c_double)
        self.st.scalar = _ptr(self.s, C.c_double)
        self.st.absorption = _ptr(self.a, C.c_double)
        self.st.species = _ptr(self.sp, C.c_uint8)
        self.st.rgb = _ptr(self.rgb, C.c_double)


def check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def frame(pose):
    out = np.zeros(13, np.float64)
    check(lib().sr_frame(C.byref(camera(pose)), _ptr(out, C.c_double)), "sr_frame")
    return out


def project(ps: Particles, pose, prm: _Params):
    out = (Proj * max(ps.st.n, 1))()
    check(lib().sr_project(C.byref(ps.st), C.byref(camera(pose)), C.byref(prm), out), "sr_project")
    return out


def scalar_range(ps: Particles, n_species, log10):
    lo = np.zeros(n_species)
    hi = np.zeros(n_species)
    check(lib().sr_scalar_range(C.byref(ps.st), n_species, int(log10), _ptr(lo, C.c_double),
                                _ptr(hi, C.c_double)), "sr_scalar_range")
    return lo, hi


def render(ps: Particles, pose, prm: _Params) -> np.ndarray:
    out = np.zeros((pose.height, pose.width, 3), np.float64)
    check(lib().sr_render(C.byref(ps.st), C.byref(camera(pose)), C.byref(prm),
                          _ptr(out, C.c_double)), "sr_render")
    return out


def render_brute(ps: Particles, pose, prm: _Params, truncate=True) -> np.ndarray:
    out = np.zeros((pose.height, pose.width, 3), np.float64)
    check(lib().sr_render_brute(C.byref(ps.st), C.byref(camera(pose)), C.byref(prm),
                                int(truncate), _ptr(out, C.c_double)), "sr_render_brute")
    return out


def render_back_to_front(ps: Particles, pose, prm: _Params) -> np.ndarray:
    out = np.zeros((pose.height, pose.width, 3), np.float64)
    check(lib().sr_render_sorted_back_to_front(C.byref(ps.st), C.byref(camera(pose)),
                                               C.byref(prm), _ptr(out, C.c_double)),
          "sr_render_sorted_back_to_front")
    return out


def record_box(rec_row, nu, width, height):
    r = np.ascontiguousarray(rec_row, dtype=np.float32)
    v = [C.c_int32() for _ in range(4)]
    ok = lib().sr_record_box(_ptr(r, C.c_float), C.c_float(nu), width, height,
                             *[C.byref(x) for x in v])
    return bool(ok), tuple(x.value for x in v)


def bin_records(rec, rec2, width, height, tile, nu, bin_rule=0, by_depth=False):
    rec = np.ascontiguousarray(rec, dtype=np.float32).reshape(-1, 8)
    rec2 = None if rec2 is None else np.ascontiguousarray(rec2, dtype=np.float32).reshape(-1, 2)
    n = rec.shape[0]
    ntx = (width + tile - 1) // tile
    nty = (height + tile - 1) // tile
    counts = np.zeros(ntx * nty, np.uint32)
    offsets = np.zeros(ntx * nty + 1, np.uint32)
    npairs = C.c_int64()
    L = lib()
    check(L.sr_bin_records(n, _ptr(rec, C.c_float), _ptr(rec2, C.c_float), width, height, tile,
                           C.c_float(nu), bin_rule, int(by_depth), _ptr(counts, C.c_uint32),
                           _ptr(offsets, C.c_uint32), None, 0, C.byref(npairs)), "count")
    pairs = np.zeros(max(npairs.value, 1), np.uint32)
    check(L.sr_bin_records(n, _ptr(rec, C.c_float), _ptr(rec2, C.c_float), width, height, tile,
                           C.c_float(nu), bin_rule, int(by_depth), _ptr(counts, C.c_uint32),
                           _ptr(offsets, C.c_uint32), _ptr(pairs, C.c_uint32), pairs.shape[0],
                           C.byref(npairs)), "bin")
    return counts, offsets, pairs[: npairs.value]


def render_records(rec, rec2, width, height, mode, nu=3.0) -> np.ndarray:
    rec = np.ascontiguousarray(rec, dtype=np.float32).reshape(-1, 8)
    rec2 = None if rec2 is None else np.ascontiguousarray(rec2, dtype=np.float32).reshape(-1, 2)
    out = np.zeros((height, width, 3), np.float64)
    check(lib().sr_render_records(rec.shape[0], _ptr(rec, C.c_float), _ptr(rec2, C.c_float),
                                  width, height, mode, nu, _ptr(out, C.c_double)),
          "sr_render_records")
    return out


def expected_flux(ps: Particles, pose, prm: _Params) -> np.ndarray:
    out = np.zeros(3, np.float64)
    check(lib().sr_expected_flux(C.byref(ps.st), C.byref(camera(pose)), C.byref(prm),
                                 _ptr(out, C.c_double)), "sr_expected_flux")
    return out


def image_stats(img):
    img = np.ascontiguousarray(img, dtype=np.float64)
    flux = np.zeros(3)
    mx = np.zeros(3)
    lib().sr_image_stats(_ptr(img, C.c_double), img.shape[1], img.shape[0],
                         _ptr(flux, C.c_double), _ptr(mx, C.c_double))
    return flux, mx
