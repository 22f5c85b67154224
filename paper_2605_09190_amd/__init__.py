"""MI355X-native AQMP encoder: HIP kernels for gfx950 behind a C ABI
(include/aqmp.h) with a thin ctypes binding (``paper_2605_09190_amd.aqmp``)."""
