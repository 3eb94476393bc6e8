"""ckc: GPU-native memory-access checking of index programs on AMD MI355X.

The library itself is ``libckc.so`` (C-ABI, ``include/ckc.h``); ``ckc`` is its
Python binding and ``gen`` holds the IR builder and the seeded workloads.
Importing this package loads nothing native.
"""
