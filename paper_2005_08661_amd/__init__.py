"""MI355X-native preconditioned NCG-MLS field-map estimator (Lin & Fessler,
"Efficient Regularized Field Map Estimation in 3D MRI", arXiv 2005.08661).

The estimator runs in hand-written HIP kernels for gfx950 behind a C ABI
(include/fmap.h, libfmap.so); this package holds the thin Python binding and
the seeded synthetic-input generator.
"""
