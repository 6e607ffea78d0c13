"""MI355X (gfx950) Scheduled Relaxation Jacobi solver with the data-driven
scheme selector of Islam & Wang (arXiv 2011.06636).

The solver lives in the HIP library libsrj.so (C ABI: include/srj.h);
``abi`` is its ctypes binding and ``solver.Solver`` a PyTorch-facing wrapper
that supplies device memory and streams.
"""
from . import abi  # noqa: F401

__all__ = ["abi", "solver"]
