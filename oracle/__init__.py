"""Plain FP64 CPU oracle for FastPI (Jung & Sael, arXiv 2011.04235).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. The product path (the HIP library and
its Python binding) never imports, calls or links anything from here, and this
package imports nothing from the product.
"""
from .reorder import Reordering, reorder, hub_count  # noqa: F401
from .fastpi import (  # noqa: F401
    target_rank, split_blocks, block_svd, row_update, column_update, fastpi_svd,
    pinv_apply, sigma_pinv, recon_error, ls_residual, orthonormality_error, OracleResult,
)
from .evaluate import (  # noqa: F401
    labels_dense, pinv_apply_sparse, row_scores, rank_k, precision_at_k, topk_hits, p_at_k,
)
from .randomized import (  # noqa: F401
    InnerSolver, gaussian, philox4x32_10, rsvd_right, sign_convention, use_randomized,
)
