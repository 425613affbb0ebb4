"""DMK Stokeslet sums (prolate kernel splitting) on AMD MI355X (gfx950).

The computation lives in libdmk_stokes.so (hand-written HIP kernels behind a C
ABI, include/dmk_stokes.h); this package only marshals arguments.
"""
from ._lib import (KERNEL_STOKESLET, KERNEL_STRESSLET, METHOD_DMK, METHOD_EWALD, PREC_FP64, PREC_MIXED, DMKError, Plan, SYMBOLS, autotune, ewald_params,
                   host_tree, lib, mollifier, params, radial, radial_stresslet, residual_sum, residual_sum_noalloc,
                   residual_sum_stresslet)

__all__ = ["Plan", "DMKError", "PREC_FP64", "PREC_MIXED", "KERNEL_STOKESLET", "KERNEL_STRESSLET", "METHOD_DMK", "METHOD_EWALD", "params", "ewald_params",
           "radial", "radial_stresslet", "mollifier", "residual_sum", "residual_sum_noalloc", "residual_sum_stresslet", "lib", "SYMBOLS", "host_tree",
           "autotune"]
