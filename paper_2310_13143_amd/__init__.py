"""MI355X-native ADMM QP solver for the SQP method for ACOPF (arXiv 2310.13143).

The computation runs in the HIP library ``libacopf_admm.so`` (C ABI declared
in ``include/acopf_admm.h``); this package only marshals arguments to it,
with PyTorch providing device memory and streams.
"""
from ._abi import AcopfError, HESSIAN_PSD, HESSIAN_RAW, HESSIAN_RAW_LOCAL, SWEEP_GRAPH, SWEEP_LAUNCHES, SWEEP_PERSISTENT  # noqa: F401

__all__ = ["AcopfError", "HESSIAN_PSD", "HESSIAN_RAW", "HESSIAN_RAW_LOCAL", "SWEEP_GRAPH", "SWEEP_LAUNCHES", "SWEEP_PERSISTENT"]
