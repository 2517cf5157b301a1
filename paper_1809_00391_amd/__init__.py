"""MI355X longitudinal multi-bunch macro-particle tracker (arXiv:1809.00391).

The compute path is libmbt.so (HIP kernels for gfx950 behind the C ABI in
include/mbt.h); `tracker` is its Python binding and `workloads` holds the
parameter presets and seeded input generators.
"""
