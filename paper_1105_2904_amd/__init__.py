"""MI355X-native hot path of the site-based suspension lattice Boltzmann method.

The compute path is the HIP library ``liblbm.so`` built from ``csrc/`` (C ABI
declared in ``include/lbm.h``); ``lbm`` is its thin ctypes binding and
``workloads`` holds the seeded synthetic inputs.  Importing the package does
not load the library: the first call through ``lbm`` does, and raises if the
library has not been built.
"""
__all__ = ["lbm", "workloads"]
