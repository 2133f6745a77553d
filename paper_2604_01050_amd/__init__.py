"""MI355X-native SBQA (Simulated Bifurcation Quantum Annealing, arXiv 2604.01050).

The solver is the C-ABI library libsbqa.so (declared in include/sbqa.h): hand
written HIP kernels for gfx950 and a C++ runtime. This package is its thin
Python binding; every entry point keeps the C name (sbqa_create, sbqa_step,
sbqa_best, ...). Build the library first with ``paper_2604_01050_amd.build``;
without it the import fails, there is no CPU fallback.
"""
from ._abi import *  # noqa: F401,F403
from ._abi import (Context, SbqaError, Server, make_schedule, lib, LIB_PATH, PATHS,  # noqa: F401
                   OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EBUDGET, EAGAIN,
                   F_TERNARY, F_SIGN, F_BALLISTIC, PREC_AUTO, PREC_FP32, PREC_FP8, PREC_BF16X3, PREC_INT8, PREC_FP4,
                   JP_LINEAR, JP_PAPER, JP_TABLE, LOOP_AUTO, LOOP_STREAM, LOOP_RESIDENT,
                   JPACK_AUTO, JPACK_BYTES, REORDER_AUTO, REORDER_OFF, REORDER_ON)
