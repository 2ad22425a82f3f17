"""MI355X solver for the isogeometric curl-div problem (HIP library + thin binding).

The compute path lives in ``libcurldiv.so`` (HIP kernels for gfx950 behind the
C ABI in ``include/curldiv.h``); ``capi`` only marshals arguments to it.
"""
from . import capi  # noqa: F401

__all__ = ["capi"]
