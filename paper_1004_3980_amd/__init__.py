"""MI355X-native hot path of patch-hashing image zoom (arXiv:1004.3980).

The work runs in libzoomhash.so (HIP kernels for gfx950 behind the C-ABI in
include/zoomhash.h); `zoomhash` is its ctypes binding and `pipeline` drives a
whole workload (dictionary, tables, query, LLE, blend, back-projection).
Importing this package loads nothing; the library is loaded on first use.
"""
