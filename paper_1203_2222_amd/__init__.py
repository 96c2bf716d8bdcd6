"""MI355X-native contraction of U(1)- and SU(2)-symmetric tensors stored as
charge-sector blocks (arXiv:1203.2222's hot path).

The compute path is libsymtensor.so (HIP kernels for gfx950 behind the C-ABI
in include/symtensor.h); this package only marshals arguments.  Build the
library with ``python -m paper_1203_2222_amd.build``.
"""
from ._lib import SymError, lib  # noqa: F401
from .tensor import (Context, Graph, Hold, SymTensor, default_variant, fmove_coeff, noalloc_capacity,  # noqa: F401
                     num_variants, su2_gamma, variant_kernel, variant_name)


def __getattr__(name):
    if name in ("contract", "SymContract"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
