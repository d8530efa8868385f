"""MI355X (gfx950) Fourier bilateral filter: HIP kernels behind a C ABI
(include/fobf.h) with a thin ctypes binding.  Importing the package loads
libfobf.so and fails loudly if it has not been built."""
from .fobf import (ALGO_AUTO, ALGO_MFMA, ALGO_VALU, BF16_STAGE, FP16_STAGE, FP16X2_STAGE,
                   FP32, KMAX, RMAX, CHECK_BITS, Coef, FobfError, Server, autotune,
                   batch_workspace_size, check_take, load_check_library, effective_prec, filter, filter_batch, filter_workspace_size, filter_ws_static, fit,
                   fit_cache_clear, fit_cache_load, fit_cache_save, fit_period, fit_samples, fit_warm, Lut, last_error, lib, make_job, peak, tune_get,
                   tune_load, tune_reset, tune_save)

__all__ = ["ALGO_AUTO", "ALGO_MFMA", "ALGO_VALU", "BF16_STAGE", "FP16_STAGE", "FP16X2_STAGE",
           "FP32", "KMAX", "RMAX", "CHECK_BITS", "Coef", "FobfError", "Server", "autotune",
           "batch_workspace_size", "check_take", "load_check_library", "effective_prec", "filter", "filter_batch", "filter_workspace_size", "filter_ws_static", "fit",
           "fit_cache_clear", "fit_cache_load", "fit_cache_save", "fit_period", "fit_samples", "fit_warm", "Lut", "last_error", "lib", "make_job", "peak", "tune_get",
           "tune_load", "tune_reset", "tune_save"]
