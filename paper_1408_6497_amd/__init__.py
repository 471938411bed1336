"""MI355X geometric multigrid for the periodic Poisson problem (hot path of arXiv 1408.6497, Section 2.3).

The solver lives in libgmg.so (hand-written HIP for gfx950, C ABI in include/gmg.h);
``gmg`` is its ctypes binding.
"""
from .gmg import (Context, GmgError, GMG_FP32, GMG_FP64, LOSS_ENERGY, LOSS_RESIDUAL, load,  # noqa: F401
                  octree_balance, octree_refine_gaussians, octree_refine_sharp_layer, SpectralSolver)
