"""Runtime specialization of data-parallel kernels for AMD Instinct MI355X.

The product is ``libsj.so`` (C ABI in ``include/sj.h``); :mod:`.sj` is its
ctypes binding with the same entry-point names.
"""
from . import sj  # noqa: F401
from .sj import *  # noqa: F401,F403
