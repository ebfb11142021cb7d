"""MI355X-native Kalman-filter track finding and fitting (arXiv:1811.04141).

The hot path is the C-ABI library libmkf.so (HIP kernels for gfx950, C ABI in
include/mkf.h); `paper_1811_04141_amd.mkf` is its Python binding."""
