"""MI355X-native bulk MTGP32 generation (HIP for gfx950 behind a C ABI).

The GPU work lives in ``csrc/`` and is compiled into ``_build/libmtgp.so``;
``mtgp`` is the thin ctypes binding over its C ABI (``include/mtgp.h``).
Importing this package loads nothing; the library is loaded on first use and
every entry point fails loudly if it is missing.
"""
__all__ = ["workloads", "mtgp"]
