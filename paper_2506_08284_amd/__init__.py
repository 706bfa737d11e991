"""MI355X structure-preserving H(curl) AMG: Python binding of libhcurl_amg.so.

The binding only marshals arguments to the C ABI declared in
include/hcurl_amg.h; every step of setup and solve runs in the library's HIP
kernels.  Arrays may be numpy arrays (host memory) or torch tensors on the GPU
(device memory, passed with ``mem_space="device"``).

Importing this package loads the compiled library and raises if it is missing:
there is no CPU fallback.
"""
from .binding import (  # noqa: F401
    HCURL_OK, HCURL_EINVAL, HCURL_EHIP, HCURL_ENOMEM, HCURL_EREDUCIBLE, HCURL_ENOTSPD, HCURL_EMAXIT,
    HCURL_EUNSUPPORTED, HCURL_ESTAGNATE, HCURL_EINFEASIBLE, HCURL_NOALLOC_MAX_ROWS, LS_HIST_J, LS_HIST_NP, HcurlError, lib, library_path, EXPORTED_SYMBOLS,
    hcurl_amg_default_opts, hcurl_amg_setup, hcurl_amg_solve, hcurl_amg_solve_noalloc, hcurl_amg_vcycle, hcurl_amg_destroy,
    hcurl_amg_update, hcurl_amg_num_levels, hcurl_amg_level_info, hcurl_amg_commute_residual, hcurl_amg_curl_residual, hcurl_amg_export_csr, hcurl_amg_export_vec, hcurl_amg_stats,
    hcurl_amg_kernel_stats, hcurl_amg_reset_kernel_stats, hcurl_last_error, hcurl_error_string, Hierarchy,
    hcurl_mpnn_num_params, hcurl_mpnn_create, hcurl_mpnn_get_params, hcurl_mpnn_destroy, hcurl_amg_mpnn_sample,
    hcurl_mpnn_sample_entries, hcurl_mpnn_sample_export, hcurl_mpnn_sample_destroy, hcurl_mpnn_forward,
    hcurl_mpnn_loss_grad, hcurl_mpnn_train_step, Network, DEV_ALLOC_FN, DEV_FREE_FN,
)
