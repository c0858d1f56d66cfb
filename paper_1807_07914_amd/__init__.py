"""MI355X (gfx950) state-vector simulation of quantum circuits.

The hot path -- gate application, fused LDS tile passes, dense k-qubit
blocks on the matrix cores, FP64 reductions and sampling -- lives in the HIP
library ``libqsv.so`` behind the C ABI of ``include/qsv.h``; this package is
its thin ctypes binding (``qsv``).
"""
from .qsv import MPS, Batch, OpList, QsvError, State, lib, pauli_masks, plan_info  # noqa: F401
