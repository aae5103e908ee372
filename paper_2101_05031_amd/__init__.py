"""MI355X (gfx950) slicer for convolution-surface lattice structures.

The slicing path (binning, field, binary image, contours, adjoint, batched
persistent slicing) runs in the native library liblsl.so behind the C ABI of
include/lsl.h; this package only binds it.  Importing the package does not
load the library; the first call does, and fails if it was not built.
"""

__all__ = ["lattice_bin", "slice_field", "slice_field_stats", "slice_contours",
           "slice_field_backward", "slice_batch", "slice_autotune", "SliceField", "Bins"]


def __getattr__(name):
    if name in ("lattice_bin", "slice_field", "slice_field_stats", "slice_contours",
                "slice_field_backward", "slice_batch", "slice_autotune", "Bins"):
        from . import api
        return getattr(api, name)
    if name == "SliceField":
        from .autograd import SliceField
        return SliceField
    raise AttributeError(name)
