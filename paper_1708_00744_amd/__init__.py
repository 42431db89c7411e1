"""MI355X (gfx950) delayed Slater-determinant updates (arXiv:1708.00744).

The compute path is libdsu.so (HIP kernels behind the C ABI of include/dsu.h);
`dsu` is its ctypes binding, `inputs` the seeded synthetic input generators.
"""
from . import inputs  # noqa: F401
