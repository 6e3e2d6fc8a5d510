"""MI355X-native quasistatic beam-plasma instability solver.

The compute path is the HIP library ``libqs.so`` (C ABI in ``include/qs.h``); ``qs`` is its
ctypes binding and ``inputs`` the seeded synthetic workloads.  Importing the package does
not load the library; ``qs.lib()`` does, and raises if it has not been built.
"""
__all__ = ["qs", "inputs"]
