"""MI355X-native exact reverse k-MIPS (Simpfer, Amagata & Hara, RecSys 2021).

The compute path is the HIP library ``librkmips.so`` (C ABI declared in
``include/rkmips.h``); :mod:`paper_2110_07131_amd.rkmips` is its thin ctypes
binding.  Importing this package does not load the native library; the
binding loads it on first use and raises if it is missing.
"""
__all__ = ["datagen"]
