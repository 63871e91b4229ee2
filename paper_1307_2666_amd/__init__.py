"""MI355X-native HIF-IE (hierarchical interpolative factorization for integral
equations, Ho & Ying, arXiv 1307.2666): Python binding of the HIP library.

``factor`` builds ``F ~ A`` on the GPU (Algorithms 4.1 / 4.2, or the RSF of
Algorithm 3.1); the returned handle applies ``F``, ``F^T``, ``F^{-1}``,
``F^{-T}``.  ``matvec`` is the exact on-the-fly ``A x``.  ``diff.solve`` is
the solve as a differentiable function of ``a`` and ``f``.
"""
from ._binding import (EXPORTS, HIF_EDEVICE, HIF_EINVAL, HIF_ENOMEM, HIF_ESINGULAR, HIF_EUNSUPPORTED,  # noqa: F401
                       HIF_FP32_MIXED, HIF_FP64, HIF_OK, HIF_SOLVE_NOALLOC_MAX, Factorization, HifError, LIB_PATH, SolveGraph,
                       default_opts, diag_grad, factor, factor_batch, id_batched, load_library, lu_batched, matvec,
                       partition, tuning_get, tuning_set)
from . import diff  # noqa: F401

__all__ = ["factor", "factor_batch", "matvec", "id_batched", "partition", "diag_grad", "diff", "Factorization", "HifError",
           "load_library", "default_opts", "LIB_PATH", "EXPORTS"]
