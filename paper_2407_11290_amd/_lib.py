"""ctypes declarations of the C ABI in include/tt_cross.h.

Loading fails loudly when libttcross.so has not been built: there is no CPU
fallback for any entry point.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TT_CROSS_LIB=stamps selects the instrumented build (phase stamps, see
# tt_cross_get_stamps); the default is the normal library
LIB_PATH = os.path.join(HERE, "libttcross_stamps.so" if os.environ.get("TT_CROSS_LIB") == "stamps"
                        else "libttcross.so")

TT_MAX_D = 16
TT_MAX_RANK = 64

FN_HILBERT, FN_MAXWELL, FN_BIMAXWELL, FN_SEPSUM, FN_MAXWELL_2D2V, FN_MAXWELL_3D3V, FN_MAXWELL_IL = 1, 2, 3, 4, 5, 6, 7
PREC_AUTO, PREC_FP64, PREC_FP32 = 0, 1, 2
PIVOT_GREEDY, PIVOT_ROOK = 0, 1
OK, NOT_CONVERGED, WARN_SAMPLED_ERR = 0, 1, 2
EINVAL, ENOMEM, EDEVICE, ESINGULAR, ESTATE, EFN, EBUSY = -1, -2, -3, -4, -5, -6, -7


class Options(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("r_max", C.c_int32),
        ("precision", C.c_int32),
        ("pivot_mode", C.c_int32),
        ("n_samples", C.c_int32),
        ("grid", C.c_int32 * TT_MAX_D),
        ("tile_rows", C.c_int32),
        ("tile_cols", C.c_int32),
        ("lookahead", C.c_int32),
        ("profile", C.c_int32),
        ("stream", C.c_void_p),
        ("verify", C.c_int32),
        ("rook_split", C.c_int32),
        ("restarts", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("evaluated", C.c_int64),
        ("pivoted", C.c_int64),
        ("samples", C.c_int64),
        ("sweeps", C.c_int32),
        ("precision_used", C.c_int32),
        ("status", C.c_int32),
        ("d", C.c_int32),
        ("ranks", C.c_int32 * (TT_MAX_D + 1)),
        ("rms", C.c_double),
        ("tau", C.c_double),
        ("time_to_eps_s", C.c_double),
        ("last_best", C.c_double * TT_MAX_D),
        ("sweep_launches", C.c_int32),
        ("rook_max_rounds", C.c_int32),
        ("sweep_kernel_s", C.c_double),
        ("sweep_alg_bytes", C.c_double),
        ("new_entries", C.c_double),
        ("sweep_phase_s", C.c_double),
        ("sampled_err", C.c_double),
        ("escalated", C.c_int32),
        ("rook_long_walks", C.c_int32),
        ("restarts_used", C.c_int32),
        ("restart_cause", C.c_int32),
    ]


TILE_ROW_WORDS = 6 + 2 * TT_MAX_D  # int32 words per row of tt_tile_table


class ServerStats(C.Structure):
    _fields_ = [(name, C.c_int64) for name in ("submitted", "completed", "queued", "running", "pool_bytes",
                                                "pool_objects", "allocations")]


# name -> (restype, argtypes); every function declared in include/tt_cross.h
SIGNATURES = {
    "tt_options_default": (None, [C.POINTER(Options)]),
    "tt_cross_create": (C.c_void_p, [C.c_int, C.POINTER(C.c_int32), C.c_double, C.c_int,
                                     C.POINTER(C.c_double), C.c_int]),
    "tt_cross_set_options": (C.c_int, [C.c_void_p, C.POINTER(Options)]),
    "tt_cross_run": (C.c_int, [C.c_void_p]),
    "tt_cross_run_async": (C.c_int, [C.c_void_p, C.c_void_p]),
    "tt_cross_query": (C.c_int, [C.c_void_p]),
    "tt_cross_wait": (C.c_int, [C.c_void_p]),
    "tt_cross_set_rank_caps": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "tt_cross_get_ranks": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "tt_cross_get_tiles": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "tt_cross_get_cores": (C.c_int64, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int]),
    "tt_eval": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int]),
    "tt_cross_get_pivots": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "tt_cross_get_history": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    "tt_cross_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "tt_cross_get_stamps": (C.c_int64, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]),
    "tt_cross_sampled_error": (C.c_int, [C.c_void_p, C.c_int64, C.c_uint64, C.POINTER(C.c_double)]),
    "tt_cross_sampled_error_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_uint64, C.POINTER(C.c_double)]),
    "tt_fn_eval": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int,
                             C.c_int64, C.c_void_p, C.c_void_p, C.c_int]),
    "tt_fn_eval_f32": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int,
                                 C.c_int64, C.c_void_p, C.c_void_p, C.c_int]),
    "tt_fn_eval_last_kernel_ms": (C.c_int, [C.POINTER(C.c_double)]),
    "tt_cross_destroy": (None, [C.c_void_p]),
    "tt_batch_run": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "tt_batch_statuses": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int32)]),
    "tt_autotune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              C.POINTER(C.c_double)]),
    "tt_batch_autotune": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "tt_tile_table": (C.c_int, [C.c_void_p, C.c_int]),
    "tt_tile_table_clear": (None, []),
    "tt_server_create": (C.c_void_p, [C.c_size_t, C.c_int, C.POINTER(Options)]),
    "tt_server_submit": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.c_double, C.c_int,
                                   C.POINTER(C.c_double), C.c_int, C.c_uint64, C.POINTER(C.c_uint64)]),
    "tt_server_poll": (C.c_int, [C.c_void_p, C.c_uint64]),
    "tt_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_double)]),
    "tt_server_result": (C.c_int64, [C.c_void_p, C.c_uint64, C.POINTER(Stats), C.c_void_p, C.c_int64]),
    "tt_server_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "tt_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "tt_server_destroy": (None, [C.c_void_p]),
    "tt_last_error": (C.c_char_p, []),
}

_lib = None


def _init_torch_first():
    """torch carries its own HIP runtime; it must bring the device up before
    this library's runtime does, or torch's later initialisation fails.  Device
    pointers and streams from torch stay valid for the library either way."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load():
    """Load libttcross.so (built by __graft_entry__.build()); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    _init_torch_first()
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error():
    return load().tt_last_error().decode(errors="replace")


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(code):
    if code < 0:
        raise TTError(code, last_error())
    return code
