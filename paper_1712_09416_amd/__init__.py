"""MI355X TPC sector tracker: HIP kernels behind a C ABI (libtpcca.so).

Python here only marshals arguments; torch provides device memory and
streams.  Nothing runs on the CPU if the native library is missing: loading
raises instead.
"""
from ._lib import TRACK_DTYPE, TpcError, NativeMissing  # noqa: F401

__all__ = ["TRACK_DTYPE", "TpcError", "NativeMissing", "Tracker"]


def __getattr__(name):
    if name == "Tracker":
        from .tracker import Tracker
        return Tracker
    raise AttributeError(name)
