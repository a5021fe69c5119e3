"""MI355X real-fluid property engine: Python binding of libprops.so.

Argument marshalling only: every property computation runs in the HIP kernels of
``libprops.so`` (built by ``paper_2312_04830_amd.build``).  PyTorch supplies device memory
and streams; tensors are passed to the C ABI as raw device pointers.  The binding fails
loudly when the library is missing.
"""
from ._lib import (  # noqa: F401
    FP64, MIXED, PTY, RHOEY, Network, PropsError, Mechanism, lib, library_path, pr, status_bits,
)
