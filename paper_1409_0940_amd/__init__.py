"""MI355X block-splitting ADMM over random Fourier features.

The compute path is libbsadmm.so (HIP kernels behind the C ABI of
include/bsadmm.h); this package only binds it.  Import is cheap: the
library is loaded on first use and raises if it has not been built.
"""

from .abi import (rff_map, bsadmm_validate, bsadmm_footprint, bsadmm_setup, bsadmm_iterate,  # noqa: F401
                  bsadmm_predict, bsadmm_get_coef, bsadmm_state_size, bsadmm_export_state,
                  bsadmm_import_state, bsadmm_objective, bsadmm_destroy, make_problem,
                  BsadmmError, lib)


def Solver(*args, **kwargs):  # noqa: N802 - factory keeps torch import lazy
    from .solver import Solver as _S
    return _S(*args, **kwargs)
