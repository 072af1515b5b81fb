"""MI355X-native Green-function-preconditioned (Lippmann-Schwinger) FFT solver
for periodic linear-elastic unit cells.

The solver itself is the HIP library liblsfft.so (C ABI in include/lsfft.h);
`lsfft` is a thin ctypes binding to it, `inputs` holds the seeded synthetic
microstructure generators.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "lsfft"]
