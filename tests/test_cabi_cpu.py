"""Host-side checks of the C ABI: the gfx950 library loads on a machine without
a GPU and exports every entry point that include/splotch.h declares."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "splotch.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spl_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["spl_create", "spl_destroy", "spl_render", "spl_render_batch", "spl_project",
              "spl_bin", "spl_render_records", "spl_scalar_range", "spl_autotune",
              "spl_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1606_04427_amd import binding

    L = binding.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(binding.EXPORTS) == set(_declared())


def test_create_without_device_reports_device_error():
    from paper_1606_04427_amd import binding

    if os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"):
        pytest.skip("a GPU device node is present")
    h = C.c_void_p()
    rc = binding.lib().spl_create(0, C.byref(h))
    assert rc == binding.SPL_EDEVICE and not h.value


def test_null_arguments_are_rejected_without_a_device():
    from paper_1606_04427_amd import binding

    L = binding.lib()
    assert L.spl_create(0, None) == binding.SPL_EINVAL
    assert L.spl_render(None, None, None, None, None, None, None) == binding.SPL_EINVAL
    assert L.spl_last_error(None) == b"no context"
    L.spl_destroy(None)


def test_struct_layouts_match_header():
    """ctypes mirrors agree with the C compiler's layout of the header."""
    import subprocess
    import tempfile

    from paper_1606_04427_amd import binding as B

    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "splotch.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(spl_particles), sizeof(spl_camera), sizeof(spl_look),
         sizeof(spl_params), sizeof(spl_stats));
  printf("%zu %zu %zu %zu\n", offsetof(spl_params, k_sigma), offsetof(spl_params, large_cut),
         offsetof(spl_particles, species), offsetof(spl_stats, tile));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    sizes = [C.sizeof(B.spl_particles), C.sizeof(B.spl_camera), C.sizeof(B.spl_look),
             C.sizeof(B.spl_params), C.sizeof(B.spl_stats)]
    offs = [B.spl_params.k_sigma.offset, B.spl_params.large_cut.offset,
            B.spl_particles.species.offset, B.spl_stats.tile.offset]
    assert [int(v) for v in out] == sizes + offs


def test_params_keep_their_palettes_alive():
    """spl_params holds raw device pointers into the palette tensors, so the
    Python object must keep the palettes referenced (a temporary Palettes
    passed inline would otherwise be freed before the render reads it)."""
    import gc
    import weakref

    from paper_1606_04427_amd import binding as B

    class FakePalettes:
        def __init__(self):
            self.t = [FakeTensor()]

    class FakeTensor:
        shape = (256, 3)

        def data_ptr(self):
            return 0x1000

    pal = FakePalettes()
    ref = weakref.ref(pal)
    prm = B.make_params(1, pal, [dict(log10=1, brightness=1.0, lo=0.0, hi=1.0)])
    del pal
    gc.collect()
    assert ref() is not None
    del prm
    gc.collect()
    assert ref() is None
