"""ctypes wrapper over the FP64 CPU oracle (oracle/tt_oracle.c).

Test infrastructure only: tests, the smoke check and the benchmark's CPU
baseline call it; the product path never does.
"""
import ctypes as C

import numpy as np

from . import build as _build

FN_HILBERT, FN_MAXWELL, FN_BIMAXWELL, FN_SEPSUM, FN_MAXWELL_2D2V, FN_MAXWELL_3D3V, FN_MAXWELL_IL = 1, 2, 3, 4, 5, 6, 7

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        P = C.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.c_int, i32p, C.c_double, C.c_int, P, C.c_int, C.c_uint64, C.c_int,
                                 C.c_int]
        L.orc_destroy.argtypes = [P]
        L.orc_run.argtypes = [P]
        L.orc_set_rook.argtypes = [P, i32p, C.c_int]
        L.orc_set_rank_caps.argtypes = [P, i32p]
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_get_ranks.argtypes = [P, i32p]
        L.orc_get_pivots.argtypes = [P, C.c_int, P, P, P, P, P]
        L.orc_get_stats.argtypes = [P, f64p, i32p]
        L.orc_get_history.argtypes = [P, C.c_int, f64p, C.c_int]
        L.orc_get_rook_rounds.argtypes = [P]
        L.orc_get_gap_history.argtypes = [P, C.c_int, f64p, C.c_int]
        L.orc_get_cores.restype = C.c_int64
        L.orc_get_cores.argtypes = [P, P, C.c_int64]
        L.orc_state_tt_eval.argtypes = [P, C.c_int64, i32p, f64p]
        L.orc_tt_eval.argtypes = [C.c_int, i32p, i32p, f64p, C.c_int64, i32p, f64p]
        L.orc_sampled_error.argtypes = [P, C.c_int64, C.c_uint64, P]
        L.orc_full_error.argtypes = [P, P, P]
        L.orc_verify.argtypes = [P, C.c_int64, P]
        L.orc_superblock_residual.restype = C.c_int64
        L.orc_superblock_residual.argtypes = [P, C.c_int, P, C.c_int64, P, P]
        L.orc_matrix_residual.argtypes = [C.c_int64, C.c_int64, f64p, C.c_int, i64p, i64p]
        L.orc_fn_eval.argtypes = [C.c_int, C.c_int, i32p, P, C.c_int, C.c_int64, i32p, f64p]
        L.orc_splitmix64_draw.restype = C.c_uint64
        L.orc_splitmix64_draw.argtypes = [C.c_uint64, C.c_int64, u64p]
        L.orc_sample_indices.argtypes = [C.c_int, i32p, C.c_uint64, C.c_int64, i32p]
        L.orc_set_restarts.argtypes = [P, C.c_int, C.c_int64]
        L.orc_get_restarts.argtypes = [P, i32p, P, P]
        L.orc_pairwise_sumsq.restype = C.c_double
        L.orc_pairwise_sumsq.argtypes = [f64p, C.c_int64]
        _lib = L
    return _lib


def _params(params):
    if params is None or len(params) == 0:
        return None, 0, None
    arr = np.ascontiguousarray(params, dtype=np.float64)
    return arr.ctypes.data_as(C.c_void_p), arr.size, arr


def splitmix64(seed, count):
    out = np.zeros(count, dtype=np.uint64)
    lib().orc_splitmix64_draw(C.c_uint64(seed), count, out)
    return out


def mix64(z):
    """SplitMix64's output function; seeds the rook-mode sample streams."""
    return int(lib().orc_mix64(C.c_uint64(z)))


def sample_indices(n, seed, count):
    n = np.ascontiguousarray(n, dtype=np.int32)
    out = np.zeros((count, n.size), dtype=np.int32)
    lib().orc_sample_indices(n.size, n, C.c_uint64(seed), count, out)
    return out


def pairwise_sumsq(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_pairwise_sumsq(v, v.size)


def fn_eval(fn_id, n, idx, params=None):
    n = np.ascontiguousarray(n, dtype=np.int32)
    idx = np.ascontiguousarray(np.atleast_2d(idx), dtype=np.int32)
    out = np.zeros(idx.shape[0], dtype=np.float64)
    pp, npar, _keep = _params(params)
    st = lib().orc_fn_eval(fn_id, n.size, n, pp, npar, idx.shape[0], idx, out)
    if st != 0:
        raise ValueError(f"orc_fn_eval failed: {st}")
    return out


def matrix_residual(A, rows, cols):
    """Residual of a dense matrix after eliminating the given pivots in order."""
    A = np.array(A, dtype=np.float64, order="C")
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    st = lib().orc_matrix_residual(A.shape[0], A.shape[1], A, rows.size, rows, cols)
    if st != 0:
        raise ValueError(f"orc_matrix_residual failed: {st}")
    return A


def tt_eval(n, ranks, cores, idx):
    n = np.ascontiguousarray(n, dtype=np.int32)
    ranks = np.ascontiguousarray(ranks, dtype=np.int32)
    cores = np.ascontiguousarray(cores, dtype=np.float64)
    idx = np.ascontiguousarray(np.atleast_2d(idx), dtype=np.int32)
    out = np.zeros(idx.shape[0], dtype=np.float64)
    st = lib().orc_tt_eval(n.size, n, ranks, cores, idx.shape[0], idx, out)
    if st != 0:
        raise ValueError(f"orc_tt_eval failed: {st}")
    return out


class Oracle:
    """One TT-cross problem solved by the FP64 CPU oracle: greedy full search
    (default) or, with pivot="rook", Alg. 1 inside every subtensor block of
    `grid` (blocks per mode), its loop run until neither step moves
    (rook_iters = 0) or, as a test option, for at most rook_iters rounds."""

    def __init__(self, n, eps, fn_id, params=None, seed=0, r_max=64, n_samples=16384, pivot="greedy",
                 grid=None, rook_iters=0, rank_caps=None, restarts=0, restart_R=4096):
        self._seed = int(seed)
        self.n = np.ascontiguousarray(n, dtype=np.int32)
        self.d = int(self.n.size)
        self.fn_id = fn_id
        self.params = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        pp, npar, self._pkeep = _params(self.params)
        self.h = lib().orc_create(self.d, self.n, float(eps), fn_id, pp, npar, C.c_uint64(seed),
                                  r_max, n_samples)
        if not self.h:
            raise ValueError("orc_create rejected the problem")
        if pivot == "rook":
            g = np.ones(self.d, dtype=np.int32) if grid is None else np.ascontiguousarray(grid, dtype=np.int32)
            if lib().orc_set_rook(self.h, g, int(rook_iters)) != 0:
                raise ValueError("orc_set_rook rejected the options")
        elif pivot != "greedy":
            raise ValueError(pivot)
        if rank_caps is not None:
            if lib().orc_set_rank_caps(self.h, np.ascontiguousarray(rank_caps, dtype=np.int32)) != 0:
                raise ValueError("orc_set_rank_caps rejected the caps")
        if restarts:
            if lib().orc_set_restarts(self.h, int(restarts), int(restart_R)) != 0:
                raise ValueError("orc_set_restarts rejected the options")
        self.status = None

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def run(self):
        self.status = lib().orc_run(self.h)
        if self.status < 0:
            raise RuntimeError(f"oracle run failed: {self.status}")
        return self.status

    def ranks(self):
        r = np.zeros(self.d + 1, dtype=np.int32)
        lib().orc_get_ranks(self.h, r)
        return r

    def pivots(self, k):
        """(row tuples r_k x k, column tuples r_k x (d-k), rho, gamma, p) of unfolding k (1-based)."""
        rk = int(self.ranks()[k])
        rows = np.zeros((rk, k), dtype=np.int32)
        cols = np.zeros((rk, self.d - k), dtype=np.int32)
        rho = np.zeros(rk, dtype=np.int64)
        gam = np.zeros(rk, dtype=np.int64)
        piv = np.zeros(rk, dtype=np.float64)
        lib().orc_get_pivots(self.h, k, rows.ctypes.data, cols.ctypes.data, rho.ctypes.data,
                             gam.ctypes.data, piv.ctypes.data)
        return rows, cols, rho, gam, piv

    def stats(self):
        out = np.zeros(7, dtype=np.float64)
        i0 = np.zeros(self.d, dtype=np.int32)
        lib().orc_get_stats(self.h, out, i0)
        return {"rms": out[0], "tau": out[1], "evaluated": int(out[2]), "pivoted": int(out[3]),
                "sweeps": int(out[4]), "min_rel_gap": out[5], "status": int(out[6]), "i0": i0}

    def restart_info(self):
        """Restarts after false convergence: {"used", "cause" (0 none, 1
        restarts used up, 2 no usable sample), "err" (the last check's error,
        -1 if none), "seeds" (the points added to i0, in order)}."""
        out = np.zeros(3, dtype=np.int32)
        e = C.c_double()
        pts = np.zeros((8, self.d), dtype=np.int32)
        lib().orc_get_restarts(self.h, out, C.byref(e), pts.ctypes.data)
        return {"used": int(out[0]), "cause": int(out[1]), "err": e.value, "seeds": pts[:int(out[2])].copy()}

    def rook_rounds(self):
        """Most rounds of Alg. 1's loop any block search took (rook mode)."""
        return int(lib().orc_get_rook_rounds(self.h))

    def gap_history(self, k):
        """Per sweep of unfolding k: (best - runner-up) / best of the search."""
        cap = 4096
        out = np.zeros(cap, dtype=np.float64)
        m = lib().orc_get_gap_history(self.h, k, out, cap)
        return out[:m].copy()

    def history(self, k):
        cap = 4096
        out = np.zeros(cap, dtype=np.float64)
        m = lib().orc_get_history(self.h, k, out, cap)
        return out[:m].copy()

    def cores_flat(self):
        m = lib().orc_get_cores(self.h, None, 0)
        out = np.zeros(m, dtype=np.float64)
        lib().orc_get_cores(self.h, out.ctypes.data, m)
        return out

    def cores(self):
        flat = self.cores_flat()
        r = self.ranks()
        res, off = [], 0
        for k in range(self.d):
            sz = int(r[k]) * int(self.n[k]) * int(r[k + 1])
            res.append(flat[off:off + sz].reshape(int(r[k]), int(self.n[k]), int(r[k + 1])))
            off += sz
        return res

    def tt_eval(self, idx):
        idx = np.ascontiguousarray(np.atleast_2d(idx), dtype=np.int32)
        out = np.zeros(idx.shape[0], dtype=np.float64)
        lib().orc_state_tt_eval(self.h, idx.shape[0], idx, out)
        return out

    def fn(self, idx):
        return fn_eval(self.fn_id, self.n, idx, self.params)

    def sampled_error(self, R=1_000_000, seed=None):
        e = C.c_double()
        s = self._seed_plus_one() if seed is None else seed
        st = lib().orc_sampled_error(self.h, R, C.c_uint64(s), C.byref(e))
        if st != 0:
            raise RuntimeError(st)
        return e.value

    def verify(self, R):
        """The final guard: sampled error over R indices of stream seed + 1;
        a converged run whose error exceeds eps gets status 2 (sampled-error
        warning).  Returns (status, error)."""
        e = C.c_double()
        st = lib().orc_verify(self.h, R, C.byref(e))
        if st < 0:
            raise RuntimeError(st)
        self.status = st
        return st, e.value

    def _seed_plus_one(self):
        return (self._seed + 1) & 0xFFFFFFFFFFFFFFFF

    def full_error(self):
        e, mx = C.c_double(), C.c_double()
        st = lib().orc_full_error(self.h, C.byref(e), C.byref(mx))
        if st != 0:
            raise RuntimeError(st)
        return e.value, mx.value

    def superblock_residual(self, k):
        nr, nc = C.c_int64(), C.c_int64()
        m = lib().orc_superblock_residual(self.h, k, None, 0, C.byref(nr), C.byref(nc))
        out = np.zeros(m, dtype=np.float64)
        lib().orc_superblock_residual(self.h, k, out.ctypes.data, m, C.byref(nr), C.byref(nc))
        return out.reshape(nr.value, nc.value)
