"""MI355X-native tile-low-rank Matern log-likelihood (arXiv 2402.09356 hot path).

The compute path is the HIP library ``libtlrmle.so`` (gfx950); this package
only marshals arguments to its C ABI (``include/tlrmle.h``).  Device memory and
streams come from PyTorch tensors.  There is no CPU fallback: importing the
binding fails loudly when the library has not been built.
"""
from .binding import (  # noqa: F401
    ORDERINGS, TlrError, Plan, lib, reorder, apply_perm, diag_gemm, diag_svd,
    status_name,
)

__all__ = ["ORDERINGS", "TlrError", "Plan", "lib", "reorder", "apply_perm", "diag_gemm", "diag_svd",
           "status_name"]
