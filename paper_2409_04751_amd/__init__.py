"""MI355X (gfx950) fisheye Gaussian-splatting rasterizer (Fisheye-GS hot path).

The compute lives in libfgs.so (HIP kernels behind the C ABI of
include/fgs.h); this package holds its ctypes binding, PyTorch-facing helpers
and the seeded synthetic workloads.
"""
from . import synth  # noqa: F401  (input generators; no GPU needed)

__all__ = ["synth", "render", "_lib"]
