"""MI355X-native operator-split multicellular stochastic simulation.

The compute path lives in ``libtissue.so`` (hand-written HIP for gfx950
behind the C-ABI declared in ``include/tissue.h``); :mod:`.tissue` is its
ctypes binding.  Importing this package loads nothing; importing
:mod:`.tissue` loads the library and raises if it is missing.
"""
__all__ = ["workloads"]
