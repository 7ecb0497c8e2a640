"""MI355X-native evaluation of the volume-potential hot path (arXiv 2203.05933).

The compute lives in libvp.so (HIP kernels for gfx950 behind the C ABI of
include/vp.h); `paper_2203_05933_amd.vp` is its thin Python binding, imported
on first use.
"""
import importlib

__all__ = ["vp"]


def __getattr__(name):
    if name == "vp":
        return importlib.import_module(".vp", __name__)
    raise AttributeError(name)
