"""MI355X-native space-time BIEM convolution (FDP=H-matrices, 2D anti-plane).

The compute path is the HIP library libbie.so (C ABI in include/bie.h);
`binding` is its ctypes wrapper.  PyTorch only provides device memory and
streams to callers.
"""
from . import binding  # noqa: F401

__all__ = ["binding"]
