"""Dense nonnegative CP (NNCP) by alternating updates on AMD MI355X (gfx950).

The computation lives in ``libnncp.so`` (hand-written HIP kernels behind the
C ABI of ``include/nncp.h``); this package is its ctypes binding.  Importing
the binding fails loudly if the library has not been built.
"""
from .binding import (  # noqa: F401
    CPLoss, Context, NNCPError, NNCP_ADMM, NNCP_BF16, NNCP_BPP, NNCP_F16, NNCP_F32, NNCP_F64, NNCP_HALS, NNCP_MU,
    NNCP_NES, NNCP_NES_OUTER,
    EXPORTS, LIB_PATH, check_problem, lib, nncp_cp_loss, nncp_destroy, nncp_gemm_path, nncp_grad, nncp_gram,
    nncp_hadamard, nncp_init, nncp_mttkrp, nncp_pgd, nncp_set_factors, nncp_split, nncp_sweep,
    nncp_update_hals, nncp_update_mu, nncp_workspace_size, nncp_timers_enable, nncp_timers_read,
    nncp_sweep_capture, nncp_update_bpp, nncp_update_admm, nncp_update_nes, nncp_mttkrp_noalloc,
    NNCP_NOALLOC_SCRATCH_BYTES, nncp_gemm_plan, nncp_read_probe, nncp_uses_fused_grad,
    nncp_factors_changed,
)
