"""MI355X (gfx950) SIMP minimum-compliance hot path (Ferrari & Sigmund,
arXiv:2005.05436): C-ABI library libtopt.so of hand-written HIP kernels and a
thin ctypes binding with the same entry-point names."""
from . import _lib
from ._lib import (TO_F32, TO_F64, TO_FILTER_ADJ, TO_FILTER_ADJ2, TO_FILTER_FWD, TO_OP_ASSEMBLED,
                   TO_OP_MATFREE, ToError, load)

__all__ = ["_lib", "load", "ToError", "TO_F32", "TO_F64", "TO_FILTER_FWD", "TO_FILTER_ADJ",
           "TO_FILTER_ADJ2", "TO_OP_ASSEMBLED", "TO_OP_MATFREE"]
