"""MI355X (gfx950) state-vector gate engine for the method of arXiv 2303.00123.

The compute path is libqsv.so (HIP kernels behind the C ABI in include/qsv.h);
this package is its Python binding.  Nothing here computes amplitudes.
"""
from .qsv import (  # noqa: F401
    QSV_C64, QSV_C128, FLAG_NO_FUSE, FLAG_FORWARD, FLAG_CAPTURE_GRAPH, FLAG_TUNE, FLAG_FROM_ZERO,
    Context, State, BatchSpec, QsvError, adjoint, plan_circuit, plan_fused, jit_source, lib, marshal_gates,
    observable_arrays, EXPORTS,
)
