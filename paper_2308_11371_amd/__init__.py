"""MI355X (gfx950) ROM-based inexact FETI-DP for lattice structures.

The compute path is libifeti.so (hand-written HIP, C ABI in include/ifeti.h);
`ifeti` is its ctypes binding.  Build the library with
`python -m paper_2308_11371_amd.build`.
"""
from . import ifeti  # noqa: F401
