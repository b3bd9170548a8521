"""MI355X (gfx950) implementation of the SZx block-wise error-bounded lossy
compressor (arXiv 2201.13020): HIP kernels behind the C ABI of include/szx.h,
and a thin ctypes binding in ``szx``."""
__all__ = ["szx", "synth"]
