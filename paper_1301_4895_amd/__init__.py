"""MI355X (gfx950) implementation of the recursive multibaryon contraction
method of Guenther, Toth and Varnhorst (arXiv:1301.4895).

The method runs in libmbcontract.so (C ABI in include/mbcontract.h): a host
term-list builder and HIP kernels for blocks and the recursion.  This package
only marshals arguments (``binding``) and allocates device buffers with
PyTorch (``runner``).
"""
from .binding import (MB_C64, MB_C128, MB_FP64, MB_MIXED, MB_MIXED_F32B, MBError, TermList, contract_correlator,
                      make_blocks, problem, workspace_query)
from .runner import Runner

__all__ = ["TermList", "Runner", "MBError", "problem", "workspace_query", "make_blocks",
           "contract_correlator", "MB_FP64", "MB_MIXED", "MB_MIXED_F32B", "MB_C64", "MB_C128"]
