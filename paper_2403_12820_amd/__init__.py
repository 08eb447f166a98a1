"""MI355X (gfx950) library for the physics-embedded CNN cloth method (arXiv 2403.12820).

The compute path is libpecnn.so (HIP kernels behind the C ABI of include/pecnn.h);
`_lib` is its ctypes binding, `inputs` the seeded synthetic scene generator,
`train` and `bench` drivers sit on top of the binding.
"""
from . import inputs  # noqa: F401  (no GPU needed)

__all__ = ["inputs"]
