"""MI355X-native D3Q19 binary-fluid lattice-Boltzmann step (HIP, gfx950).

The computation lives in the HIP library ``liblbmi.so`` behind the C ABI of
``include/lb.h``; this package is its Python binding (``LB``) plus the
reverse-mode ``torch.autograd.Function`` (``rollout``).
"""
from ._abi import LbError, LB_FP32_DEV, LB_FP64  # noqa: F401
from .lb import LB  # noqa: F401

__all__ = ["LB", "LbError", "LB_FP64", "LB_FP32_DEV"]
