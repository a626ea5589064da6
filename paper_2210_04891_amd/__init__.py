"""MI355X (gfx950) pre-corrected-FFT loop-analysis RL extractor.

The computation lives in ``libpfft.so`` (HIP kernels + host setup, C ABI in
``include/pfft.h``); ``pfft`` is its ctypes binding.
"""
from .pfft import (Context, HostModel, extract_RL, load, PfftError, PFFT_FAR_ONLY, PFFT_NEAR_ONLY,
                   PFFT_PRECOND, PFFT_PRECOND_ONLY, PFFT_LEARNED_ONLY, EXPORTS, LIB_PATH, mlp_blob,
                   mlp_params, mlp_grad)

__all__ = ["Context", "HostModel", "extract_RL", "load", "PfftError", "PFFT_FAR_ONLY", "PFFT_NEAR_ONLY",
           "PFFT_PRECOND", "PFFT_PRECOND_ONLY", "PFFT_LEARNED_ONLY", "EXPORTS", "LIB_PATH", "mlp_blob",
           "mlp_params", "mlp_grad"]
