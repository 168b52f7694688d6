"""Exact space-time hypergraph matching (arXiv 1505.00581) on AMD MI355X.

The compute path is libstm.so (hand-written HIP kernels for gfx950 behind the
C ABI in include/stm.h); this package is its Python binding and the seeded
synthetic workloads.  Build the library with
`python -m paper_1505_00581_amd.build`.
"""
from ._binding import (EXPORTS, LIB_PATH, STM_DEVICE_PTRS, STM_EHIP, STM_EINVAL, STM_ENOMEM,
                       STM_EUNSUPPORTED, STM_K_DENSITY, STM_K_LIMIT, STM_NOALLOC_SCRATCH_BYTES, STM_OK,
                       STM_UNARY_BF16,
                       Context, DevicePoints, Plan, Pruner, StmError, Trellis, load,
                       pruner_num_params)
from .synth import Params, Points

__all__ = ["Context", "DevicePoints", "Params", "Plan", "Points", "Pruner", "Trellis", "pruner_num_params", "StmError", "load", "EXPORTS",
           "LIB_PATH", "STM_OK", "STM_EINVAL", "STM_ENOMEM", "STM_EHIP", "STM_EUNSUPPORTED",
           "STM_K_LIMIT", "STM_DEVICE_PTRS", "STM_K_DENSITY", "STM_UNARY_BF16",
           "STM_NOALLOC_SCRATCH_BYTES"]
