"""MI355X (gfx950) Splotch particle renderer.

The render pipeline (projection + colour, tile binning, splat, depth-sorted
compositing, finalisation) runs in the HIP library libsplotch_hip.so behind
the C ABI of include/splotch.h; `binding` marshals arguments to it and
`synth` draws seeded synthetic inputs.  Importing the package loads nothing;
the first binding call loads the library and raises if it is missing.
"""
from . import synth  # noqa: F401

__all__ = ["synth", "binding"]
