"""MI355X-native multi-time-step PD/FE fracture solver (arXiv 2403.03605).

The solver lives in the HIP library libmtspd.so behind the C-ABI of
include/mtspd.h; this package only marshals arguments.  Importing the package
does not touch the GPU; creating a Solver loads the library and fails loudly if
it has not been built.
"""
from ._lib import (  # noqa: F401
    COUPLED, PURE_PD, FP64, MIXED,
    PD_U, PD_V, PD_A, FE_U, FE_V, FE_A, DAMAGE, LAMBDA, PD_ALPHA, PD_MASS, FE_MASS, FE_X,
    CONSTRAINT_NODES, H, KT_PD_SUBSTEP, KT_LINK, KT_FE, KT_LAMBDA, KT_REBUILD,
    REQ_ACTIVE, REQ_DONE, MtsError, Solver, Pool, load, plan, LIB_PATH, EXPORTS,
)
