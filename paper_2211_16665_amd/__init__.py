"""MI355X implementation of fictitious-wave-domain CSEM modelling and its
adjoint gradient (Yang, arXiv 2211.16665).

The compute path is the HIP library ``lib/libfwdem.so`` (C ABI in
include/fwdem.h).  ``fwdem`` is its ctypes binding, ``autograd`` the
torch.autograd wrapper, ``inversion`` the l-BFGS driver over the library's
gradient, ``reciprocity`` the source-receiver swap (index maps only).
Importing ``Plan`` loads the library and fails if it has not been built
(python -m paper_2211_16665_amd.build).
"""
from .fwdem import FwdError, Plan, load  # noqa: F401

__all__ = ["Plan", "FwdError", "load"]
