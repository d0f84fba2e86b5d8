"""MI355X-native short-range Lennard-Jones MD hot path (gfx950 HIP behind a C ABI).

The compute lives in ``libmdgpu.so`` (built from ``csrc/``); ``binding`` holds the
ctypes marshalling layer with the same names as the C entry points.
"""
