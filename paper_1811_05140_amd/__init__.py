"""aalcsim: amplitude-aware lossy-compressed state-vector simulation on MI355X.

The compute path is the HIP library libaalcsim.so (C ABI, include/aalcsim.h);
`aalcsim` is its ctypes binding and `inputs` generates seeded circuits.
Submodules are imported lazily so that generating circuits does not load the
GPU library.
"""
__all__ = ["aalcsim", "inputs"]
