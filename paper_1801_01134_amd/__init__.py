"""MI355X (gfx950) library for the mask-block sparse matrix-vector product of
Bramas & Kus (beta(r,c) storage without zero padding).

The compute lives in libspc5hip.so (HIP kernels behind a C ABI declared in
include/spc5hip.h); this package is its Python binding plus the seeded input
generators in ``synth``.
"""
from . import synth  # noqa: F401
from ._binding import (CLASS_TEST_B1X8, CLASS_TEST_B2X4, MLP_N_PARAMS, N_CLASSES, SEL_INTERP,  # noqa: F401
                       SEL_MLP, Selector, class_mode, class_shape, mlp_infer, mlp_loss_grad, mlp_n_params,
                       mlp_standardizer, mlp_targets, mlp_train)
from ._binding import SPMM_AUTO, SPMM_BITS, SPMM_ROWS, CUStream, device_cu_count  # noqa: F401
from ._binding import (SHAPES, Batch, BetaMatrix, Plan, SpcError, autotune, beta_to_csr, cg,  # noqa: F401
                       csr_permute, csr_to_beta, lib, mask_bytes, matrix_features, permute_vector, plan_from,
                       rcm_order, spmm, spmv, time_spmv)
