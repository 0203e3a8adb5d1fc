"""MI355X (gfx950) library for the mask-block sparse matrix-vector product of
Bramas & Kus (beta(r,c) storage without zero padding).

The compute lives in libspc5hip.so (HIP kernels behind a C ABI declared in
include/spc5hip.h); this package is its Python binding plus the seeded input
generators in ``synth``.
"""
from . import synth  # noqa: F401
from ._binding import (MLP_N_PARAMS, SEL_INTERP, SEL_MLP, Selector, mlp_infer, mlp_loss_grad,  # noqa: F401
                       mlp_standardizer, mlp_targets, mlp_train)
from ._binding import CUStream, device_cu_count  # noqa: F401
from ._binding import (SHAPES, Batch, BetaMatrix, Plan, SpcError, autotune, beta_to_csr, cg,  # noqa: F401
                       csr_permute, csr_to_beta, lib, mask_bytes, matrix_features, permute_vector, plan_from,
                       rcm_order, spmm, spmv, time_spmv)
