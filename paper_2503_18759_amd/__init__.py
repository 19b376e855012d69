"""MI355X (gfx950) CP-ALS-QR: QR-based CP decomposition with the restructured
dimension tree and customised Q0 extrapolation of arXiv 2503.18759.

The compute path is libcpqr.so (hand-written HIP kernels behind a C ABI,
``include/cpqr.h``); :mod:`paper_2503_18759_amd.cpqr` is its ctypes binding.
"""
from .cpqr import (CpqrError, Handle, Session, check_args, cp_als_qr,  # noqa: F401
                   cp_als_qr_batched, default_handle, load_library, mlp_forward, mlp_grad,
                   mlp_train, noalloc_last_error, qr, qr_noalloc, schedule, to_device, ttm,
                   tune_cache_check, tune_cache_path)
