"""MI355X real-fluid property engine: Python binding of libprops.so.

Argument marshalling only: every property computation runs in the HIP kernels of
``libprops.so`` (built by ``paper_2312_04830_amd.build``).  PyTorch supplies device memory
and streams; tensors are passed to the C ABI as raw device pointers.  The binding fails
loudly when the library is missing.
"""
from ._lib import (  # noqa: F401
    EXEC_GPU, EXEC_MOCK, FP64, HPY, MIXED, PTY, RHOEY, ROUTE_DNN, ROUTE_PR_FP64, ROUTE_PR_MIXED, Network,
    PropsError, Mechanism, Server, diffusion, features_hpz, lib, library_path, pr, status_bits, stream_copy,
)
