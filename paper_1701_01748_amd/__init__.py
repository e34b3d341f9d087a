"""MI355X (gfx950) implementation of the per-iteration hot path of the
preconditioned primal-dual (PPD) radio-interferometric imager of Onose,
Dabbech & Wiaux (2017).

The work runs in the HIP kernels of ``libppd.so`` (C ABI in
``include/ppd.h``); ``ppd`` is its ctypes binding, ``autograd`` wraps the
operators as differentiable torch functions.
"""
from . import ppd  # noqa: F401
