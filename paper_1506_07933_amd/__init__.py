"""MI355X-native local phases of the pencil 3-D FFT (AccFFT, Sec. 2).

The transforms run in libmifft.so (hand-written HIP for gfx950, C ABI in
include/mifft.h); this package is its thin Python binding.  Importing the
package does not load the library; touching ``Plan`` and friends does, and
raises if it is not built.
"""
import importlib

__all__ = ["Plan", "PencilPlan", "SlabPlan", "BatchPlan", "MifftError"]


def __getattr__(name):
    if name in ("Plan", "PencilPlan", "SlabPlan", "MifftError"):
        return getattr(importlib.import_module(".fft", __name__), name)
    if name == "BatchPlan":
        return importlib.import_module(".batch", __name__).BatchPlan
    raise AttributeError(name)
