"""MI355X-native chunked test-time training (fast-weight MLP update/apply).

The computation runs in the HIP library libttt_hip.so (C ABI: include/ttt.h);
this package only marshals torch tensors to it.
"""
from ._lib import load, TTTError  # noqa: F401
from . import ops  # noqa: F401

__all__ = ["load", "TTTError", "ops"]
