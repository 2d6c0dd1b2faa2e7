"""MI355X-native TDGL + Poisson time-step library (FerroX, arXiv 2210.15668).

The compute path is the HIP shared library ``libferrox.so`` built from
``csrc/``; ``paper_2210_15668_amd.ferrox`` is its thin ctypes binding.
Importing this package does not load the library; ``ferrox.lib()`` does,
and raises if it is missing.
"""
__all__ = ["workloads"]
