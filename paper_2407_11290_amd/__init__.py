"""MI355X (gfx950) greedy adaptive tensor-train cross approximation.

Python binding of the C ABI in include/tt_cross.h; the work runs in the HIP
library libttcross.so, which must be built first (__graft_entry__.build()).
Importing the package does not load the library.
"""
from ._lib import (EBUSY, EDEVICE, EFN, EINVAL, ENOMEM, ESINGULAR, ESTATE, FN_BIMAXWELL,  # noqa: F401
                   FN_HILBERT, FN_MAXWELL, FN_MAXWELL_2D2V, FN_MAXWELL_3D3V, FN_MAXWELL_IL, FN_SEPSUM, LIB_PATH,
                   NOT_CONVERGED, OK, PIVOT_GREEDY, PIVOT_ROOK, PREC_AUTO, PREC_FP32, PREC_FP64, TTError,
                   WARN_SAMPLED_ERR)


def __getattr__(name):
    if name in ("TTCross", "fn_eval", "fn_eval_last_kernel_ms", "default_options", "batch_run", "Server",
                "batch_autotune", "tile_table", "tile_table_clear"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
