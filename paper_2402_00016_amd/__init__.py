"""MI355X-native Multipolynomial Monte Carlo trace estimation.

The GPU path lives in ``libmpmc.so`` (HIP for gfx950, C ABI declared in
``include/mpmc.h``); ``mpmc`` is its thin ctypes binding and ``driver`` the
host-side Monte Carlo bookkeeping.  Submodules are imported lazily so that the
input generator can be used without loading the GPU library.
"""
