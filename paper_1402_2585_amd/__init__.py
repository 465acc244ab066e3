"""MI355X-native hot path of hierarchically deflated CG (arXiv:1402.2585).

The compute lives in the HIP library libhdcg.so (built in-tree by
``paper_1402_2585_amd.build``); this package is its ctypes binding plus
small helpers that allocate device buffers with PyTorch.  Importing the
package fails loudly if the library has not been built: there is no CPU
fallback.
"""
from ._lib import (  # noqa: F401
    DWF_BF16, DWF_C64, DWF_C128, DWF_F16, DWF_NOT_CONVERGED, DWF_OK, HdcgError, cg_solve, cg_solve_mixed,
    dwf_cg_update, dwf_convert, dwf_create, dwf_create_mobius, dwf_destroy, dwf_set_hop_shape, dwf_get_hop_shape, dwf_tune_hop, dwf_release_workspace, dwf_dot, dwf_export, dwf_field_bytes,
    dwf_multishift_cg,
    dwf_import, dwf_last_error, dwf_norm2, dwf_xpay, load, mpc_apply, mpc_dag_mpc_apply,
    coarse_apply, hdcg_coarse_solve, hdcg_coarse_iterations, hdcg_mfma_tile, hdcg_coarse_solve_noalloc, hdcg_default_params, hdcg_destroy, hdcg_dims, hdcg_export_block_map,
    hdcg_export_coarse, hdcg_import_coarse, hdcg_export_ldop, hdcg_export_subspace, hdcg_ldop_setup, hdcg_mirs, hdcg_project,
    hdcg_promote, hdcg_set_params, hdcg_setup,
    hdcg_solve, hdcg_trunc_apply, hdcg_m1_interval, hdcg_chebyshev, hdcg_trunc_cg, hdcg_adef1_precondition,
)
from .fields import HDCG, FineOperator  # noqa: F401

load()
