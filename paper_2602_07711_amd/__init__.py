"""MI355X-native compact-Helmholtz solver: EigT/PFFT-preconditioned (F)GMRES on hand-written HIP kernels.

The compute path lives in libhelm.so (C ABI, include/helm.h); `helm` is its ctypes binding.
"""
from .helm import (  # noqa: F401
    Cnn,
    HelmError,
    helm_batch_create,
    helm_batch_destroy,
    helm_autotune,
    helm_batch_solve,
    helm_gemm_config,
    helm_destroy,
    helm_eig1d,
    helm_gmres_solve,
    helm_matvec,
    helm_precond_apply,
    helm_precond_apply_noalloc,
    helm_profile_enable,
    helm_profile_read,
    helm_rhs,
    helm_scale_guess,
    helm_setup,
    lib,
)
