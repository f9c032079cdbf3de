"""lqtrace on MI355X: deflated Hutchinson estimation of trace(A^{-1}) for the Wilson-Dirac
operator (Romero, Stathopoulos, Orginos, arXiv:1909.12234), as a HIP library for gfx950
behind a C-ABI (include/lqtrace.h) with this thin Python binding."""
from .lqtrace import (  # noqa: F401
    A, A_DAG, A_G5, G5_A, F64, F32, F16, BF16, OBLIQUE_G5, ORTH,
    LQT_OK, LQT_EINVAL, LQT_ENOMEM, LQT_EHIP, LQT_ENOTCONV, LQT_ENOTUNITARY, LQT_ESTATE, LQT_ENAN,
    NET_FEATURES, WEIGHT_COUNT, Basis, Context, LqtError, lib, exported_symbols,
)
