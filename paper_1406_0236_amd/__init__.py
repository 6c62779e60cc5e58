"""MI355X (gfx950) solver for multibody acoustic scattering off bodies of
revolution: block-diagonal-preconditioned GMRES on the combined-field BIE
(Hao, Martinsson, Young, arXiv 1406.0236), hand-written HIP behind a C ABI
(include/axs.h).  This package is the thin Python binding."""
from ._lib import (FP32, FP64, SOLVE_CERTIFY, SOLVE_FP64, SOLVE_MIXED, SOLVE_RESTART_INNER, SOLVE_UNPRECONDITIONED, AxsError, Context,  # noqa: F401
                   LIB_PATH, Mlp, load, mlp_predict, mlp_train, warm_start_decode, warm_start_encode,
                   warm_start_size)
