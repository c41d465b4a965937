"""MI355X-native nested Krylov sign function sgn(gamma5 Dw(mu)) x.

The compute path is the HIP library ``libnk.so`` (C ABI in include/nk.h);
``paper_0910_2918_amd.nk`` is its ctypes binding.
"""
from . import nk  # noqa: F401

__all__ = ["nk"]
