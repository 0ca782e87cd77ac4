"""MI355X-native FIZI/Mouse pipeline (arXiv 1907.04393): HIP kernels behind a
C ABI (include/fizi.h) and a thin ctypes binding."""
