"""Wilson-Dirac hopping term (Eq. 3 of arXiv:0710.2442) and solvers on MI355X.

Thin Python binding of ``libwd.so`` (see ``include/wd.h``).  Functions carry
the C names and only marshal arguments: fields are torch device tensors
(uint8 buffers of ``wd_field_bytes`` bytes, or complex128 canonical arrays for
pack/unpack), passed by pointer; every computation runs in the library's HIP
kernels.  There is no fallback: if the library is missing, importing this
package raises.
"""
from ._lib import (  # noqa: F401
    LIB_PATH,
    WD_BF16,
    WD_DAGGER,
    WD_TUNE_CACHED_STORE,
    WD_EVEN,
    WD_F16,
    WD_F32,
    WD_F64,
    WD_FULL,
    WD_ODD,
    WD_SOLVER_CG,
    WD_SOLVER_DEFECT_CG,
    WD_SOLVER_FGCR,
    PRECS,
    WdError,
    Gauge,
    lib,
    wd_caxpy,
    wd_convert,
    wd_cdot,
    wd_dslash,
    wd_dslash_ex,
    wd_dslash_mrhs,
    wd_field_bytes,
    wd_gauge_create,
    wd_gauge_destroy,
    wd_new_field,
    wd_norm2,
    wd_solve,
    wd_solve_mrhs,
    wd_solve_batch,
    wd_solve_params_default,
    wd_spinor_pack,
    wd_spinor_unpack,
    wd_status_string,
    wd_vh_pad,
    wd_tune_dslash,
    wd_set_dslash_variant,
    wd_get_dslash_variant,
    Ptc,
    ptc_weights_to_flat,
    ptc_flat_to_weights,
    wd_ptc_create,
    wd_ptc_set_weights,
    wd_ptc_get_weights,
    wd_ptc_apply,
    wd_ptc_loss_grad,
    wd_ptc_train_step,
)
