"""MI355X (gfx950) image-plane single-pulse search: de-dispersion, boxcar, S/N, candidates.

The compute path is the HIP library `libnsfrb.so` built from `csrc/`; the
Python module `nsfrb` binds its C ABI with ctypes. `synth` generates seeded
synthetic input cubes.
"""
