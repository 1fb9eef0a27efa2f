"""MI355X-native condensed-space interior-point method for polar ACOPF.

The compute path lives in the HIP/C++ shared library ``libopf.so`` (built by
``paper_2307_16830_amd.build``); :mod:`paper_2307_16830_amd.opf` is a thin
ctypes binding over its C ABI.  :mod:`paper_2307_16830_amd.gridgen` produces
seeded synthetic instances.  Submodules are imported lazily so that the input
generator can be used without loading the native library.
"""
__all__ = ["gridgen", "opf"]
