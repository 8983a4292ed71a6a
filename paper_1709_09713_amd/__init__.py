"""MI355X (gfx950) compressible Navier-Stokes residual + low-storage RK3.

Python face of the C ABI in ``include/ns_tgv.h`` (same names, argument
marshalling only) plus ``Solver``, a convenience holder of one state and
its workspace in device memory.  The hot path runs entirely in the HIP
kernels of ``libns_tgv.so``; there is no CPU fallback.
"""
from ._native import (ALGOS, DIAG_NAMES, EXPORTS, NS_ALGO_FUSED, NS_ALGO_SOME, NS_ALGO_STORED,  # noqa: F401
                      NS_ERR_ARG, NS_ERR_DEVICE, NS_ERR_NONFINITE, NS_ERR_SHAPE,
                      NS_ERR_UNSUPPORTED, NS_ERR_WORKSPACE, NS_FP32_STORE, NS_FP64, NS_OK,
                      PRECS, TILES, NativeError, diagnostics, lib, make_params,
                      ns_get_fused_config, ns_get_fused_order, ns_residual, ns_set_fused_config, ns_set_fused_order, ns_stage_stream, ns_state_bytes,
                      ns_workspace_bytes, rk3_step, rk3_step_noalloc, ns_noalloc_scratch_bytes,
                      status_string, tgv_init)
from ._native import (ns_batch_add, ns_batch_create, ns_batch_destroy, ns_batch_info,  # noqa: F401
                      ns_batch_poll, ns_batch_remove, ns_batch_set_graphs, ns_batch_step)
from .batch import Batch  # noqa: F401
from .solver import Solver  # noqa: F401
