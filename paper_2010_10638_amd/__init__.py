"""Sparse Tucker decomposition (HOOI with QR column pivoting) on AMD MI355X (gfx950).

The computation lives in the HIP library ``lib/libsptucker.so`` (C ABI: include/sptucker.h);
``binding`` marshals torch tensors into it.
"""
from .binding import (  # noqa: F401
    EXPORTS, LIB_PATH, TuckerError, core_fit, core_fit_static, hosvd_init, hooi_run, hooi_sweep, load_library, qrp_gaps, qrp_update, reconstruct, ttmc_kernel, svd_info, svd_update,
    ttmc_adjoint, ttmc_memo_pair, ttmc_mode, tucker_free, tucker_profile, tucker_profile_read, tucker_get_csf, tucker_get_info,
    tucker_init,
)
from .autograd import TuckerCompletionLoss, completion_loss  # noqa: F401
