"""MI355X-native ray-MRF loopy belief propagation (MRFMap, arXiv 2006.03512).

The compute path is ``libmrf.so`` (hand-written gfx950 HIP kernels behind the
C ABI of ``include/mrf.h``); ``RayMRF`` and ``MRFInfer`` marshal torch device
tensors into it.  ``scenes`` generates seeded synthetic depth scenes.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes", "RayMRF", "MRFInfer", "lib"]


def __getattr__(name):
    if name in ("RayMRF", "MRFInfer"):
        from . import mrf
        return getattr(mrf, name)
    if name == "lib":
        from ._lib import lib
        return lib
    raise AttributeError(name)
