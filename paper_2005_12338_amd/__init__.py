"""MI355X-native RS-SRI-GF2 hot path (range-separated stochastic RI, GF2).

The HIP library ``libgf2.so`` (built from ``csrc/`` by ``build.py``) holds
every kernel; ``gf2`` is its ctypes binding.  Importing this package does
not load the library; ``gf2.load()`` / ``gf2.Context`` do, and raise if it
has not been built.
"""
__all__ = ["gf2", "build"]
