"""MI355X (gfx950) PbP-QLP: projection-based partial QLP low-rank factorization.

The computation lives in libpbpqlp.so (HIP kernels behind the C ABI of
include/pbpqlp.h); this package only binds it.  See pbpqlp.py.
"""
from .pbpqlp import (Batch, Factorizer, Info, Model, PbpqlpError, PLANS, factor, factor_auto, factor_sketch,
                     library, matmul, omega, orth, probe, probe_features, reconstruct, residual, small_qr,
                     tune_factor, tune_lookup, tune_clear, tune_save, tune_load, workspace_size)

__all__ = ["Batch", "Factorizer", "Info", "Model", "PbpqlpError", "PLANS", "factor", "factor_auto", "factor_sketch",
           "library", "matmul", "omega", "orth", "probe", "probe_features", "reconstruct", "residual", "small_qr", "tune_factor",
           "tune_lookup", "tune_clear", "tune_save", "tune_load",
           "workspace_size"]
