"""fdtdb: the FDTD-Bath time step (arXiv 2505.23963) on AMD MI355X (gfx950).

The compute path is libfdtdb.so (hand-written HIP kernels behind the C-ABI
of include/fdtdb.h); this package is its thin ctypes binding.
"""
from .fdtdb import (BC_CLOSED, BC_PERIODIC, BC_PML, F32, F64, Batch, FdtdbError, Grid, Trainer,  # noqa: F401
                    bath_params, closure_weights, lib, set_allocator, torch_allocator)

__all__ = ["Grid", "Batch", "Trainer", "FdtdbError", "bath_params", "closure_weights", "lib", "set_allocator",
           "torch_allocator"]
