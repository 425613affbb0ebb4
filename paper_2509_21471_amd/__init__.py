"""DMK Stokeslet sums (prolate kernel splitting) on AMD MI355X (gfx950).

The computation lives in libdmk_stokes.so (hand-written HIP kernels behind a C
ABI, include/dmk_stokes.h); this package only marshals arguments.
"""
from ._lib import (PREC_FP64, PREC_MIXED, DMKError, Plan, SYMBOLS, autotune, host_tree, lib, mollifier, params,
                   radial, residual_sum)

__all__ = ["Plan", "DMKError", "PREC_FP64", "PREC_MIXED", "params", "radial", "mollifier", "residual_sum",
           "lib", "SYMBOLS", "host_tree", "autotune"]
