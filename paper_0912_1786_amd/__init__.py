"""MI355X-native Tree+SPH per-step force engine (EvoL, arXiv:0912.1786).

The compute path is the HIP library ``libtsph.so`` behind the C ABI declared
in ``include/tsph.h``; :mod:`paper_0912_1786_amd.tsph` is its thin ctypes
binding.  :mod:`paper_0912_1786_amd.inputs` draws seeded initial conditions.
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["inputs", "tsph"]
