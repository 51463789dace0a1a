"""MI355X-native SIPF-W time step: HIP kernels for gfx950 behind the C-ABI library libsipf.

Submodules are imported lazily: ``workloads`` builds seeded inputs without touching the GPU
library, ``sipf`` is the ctypes binding of libsipf.so (it raises if the library is missing).
"""
