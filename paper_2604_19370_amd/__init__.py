"""MI355X-native quasi-implicit IGA-ADS wildfire stepper.

The compute path is the HIP library ``libiga.so`` (C ABI, ``include/iga.h``);
``paper_2604_19370_amd.iga`` is its thin ctypes binding.  Importing this package
loads nothing: the library is loaded on first use and a missing library is an
error, never a fallback.
"""
__all__ = ["inputs", "iga"]
