"""MI355X matrix-free finite-strain hyperelasticity with geometric multigrid.

The compute path is libmfh.so (HIP kernels for gfx950 behind the C ABI of
include/mfh.h); ``paper_1904_13131_amd.mfh`` is its thin ctypes binding.
"""
from .mfh import (F32, F64, QP_CACHE_F, QP_CACHE_T2, QP_CACHE_T4, QP_RECOMPUTE, SCATTER_ATOMIC,  # noqa: F401
                  SCATTER_COLOR, SCATTER_AUTO, SCATTER_ELEMENT, SCATTER_TILE, LEVEL_FIELD_NODAL, LEVEL_FIELD_VERTEX,
                  COARSE_DIRECT, COARSE_CHEBYSHEV, LAW_NEO_HOOKE, LAW_MOONEY_RIVLIN,
                  Batch, MfhError, Problem, dense_inverse, lib, make_desc, workspace_size)
