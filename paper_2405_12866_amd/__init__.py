"""MI355X (gfx950) implementation of the QFactor-Sample instantiation hot path
(arXiv 2405.12866): HIP kernels and host runtime in libqfs_hip.so behind the C ABI of
include/qfs.h, with a thin ctypes binding in ``qfs``."""
__all__ = ["qfs", "inputs", "build"]
