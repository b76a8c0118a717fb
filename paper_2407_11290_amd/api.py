"""Python view of the C ABI: argument marshalling only, every step runs in the
HIP library (libttcross.so)."""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import Options, Stats, check, load


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _params_ptr(params):
    if params is None or len(params) == 0:
        return None, 0, None
    arr = np.ascontiguousarray(params, dtype=np.float64)
    return arr.ctypes.data_as(C.POINTER(C.c_double)), int(arr.size), arr


def default_options():
    o = Options()
    load().tt_options_default(C.byref(o))
    return o


def fn_eval(fn_id, n, idx, params=None, fp32=False):
    """Generating function at m multi-indices, evaluated on the GPU in FP64
    (tt_fn_eval) or, with fp32=True, in the FP32 arithmetic of FP32 sweeps
    (tt_fn_eval_f32).

    idx: numpy (m, d) int32 on the host, or a torch int32 CUDA tensor (the
    result is then a torch CUDA tensor)."""
    n = _i32(n)
    pp, npar, _keep = _params_ptr(params)
    L = load()
    fn = L.tt_fn_eval_f32 if fp32 else L.tt_fn_eval
    if hasattr(idx, "is_cuda") and idx.is_cuda:
        import torch
        idx = idx.contiguous()
        out = torch.empty(idx.shape[0], dtype=torch.float32 if fp32 else torch.float64, device=idx.device)
        check(fn(fn_id, n.size, n.ctypes.data_as(C.POINTER(C.c_int32)), pp, npar,
                 idx.shape[0], C.c_void_p(idx.data_ptr()), C.c_void_p(out.data_ptr()), 1))
        return out
    idx = _i32(np.atleast_2d(idx))
    out = np.zeros(idx.shape[0], dtype=np.float32 if fp32 else np.float64)
    check(fn(fn_id, n.size, n.ctypes.data_as(C.POINTER(C.c_int32)), pp, npar, idx.shape[0],
             idx.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p), 0))
    return out


def fn_eval_last_kernel_ms():
    """Device time (ms) of the kernel of the last completed fn_eval call, from
    events attached to its dispatch (tt_fn_eval_last_kernel_ms)."""
    ms = C.c_double()
    check(load().tt_fn_eval_last_kernel_ms(C.byref(ms)))
    return ms.value


def _stats_dict(s, d):
    return {
        "evaluated": s.evaluated, "pivoted": s.pivoted, "samples": s.samples, "sweeps": s.sweeps,
        "precision_used": s.precision_used, "status": s.status,
        "ranks": list(s.ranks)[: d + 1], "rms": s.rms, "tau": s.tau,
        "time_to_eps_s": s.time_to_eps_s, "last_best": list(s.last_best)[: max(d - 1, 0)],
        "sweep_launches": s.sweep_launches, "sweep_kernel_s": s.sweep_kernel_s,
        "sweep_alg_bytes": s.sweep_alg_bytes,
        "new_entries": s.new_entries, "sweep_phase_s": s.sweep_phase_s,
        "sampled_err": s.sampled_err, "escalated": s.escalated,
        "rook_max_rounds": s.rook_max_rounds, "rook_long_walks": s.rook_long_walks,
        "restarts_used": s.restarts_used, "restart_cause": s.restart_cause,
    }


class TTCross:
    """One cross approximation problem (a tt_cross_h handle)."""

    def __init__(self, n, eps, fn_id, params=None, seed=0, r_max=64, precision=_lib.PREC_AUTO,
                 n_samples=16384, grid=None, tile_rows=0, tile_cols=0, lookahead=2, profile=0,
                 stream=None, verify=-1, pivot=_lib.PIVOT_GREEDY, rook_split=0, restarts=0):
        L = load()
        self.n = _i32(n)
        self.d = int(self.n.size)
        self.fn_id = fn_id
        self.params = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        pp, npar, self._pkeep = _params_ptr(self.params)
        self.h = L.tt_cross_create(self.d, self.n.ctypes.data_as(C.POINTER(C.c_int32)), float(eps), fn_id,
                                   pp, npar)
        if not self.h:
            raise _lib.TTError(_lib.EINVAL, _lib.last_error())
        o = default_options()
        o.seed = seed
        o.r_max = r_max
        o.precision = precision
        o.n_samples = n_samples
        if grid is not None:
            for j, c in enumerate(grid):
                o.grid[j] = int(c)
        o.tile_rows = tile_rows
        o.tile_cols = tile_cols
        o.lookahead = lookahead
        o.profile = profile
        o.verify = verify
        o.pivot_mode = pivot
        o.rook_split = rook_split
        o.restarts = restarts
        if stream is not None:
            o.stream = C.c_void_p(getattr(stream, "cuda_stream", stream))
        check(L.tt_cross_set_options(self.h, C.byref(o)))
        self.status = None

    def close(self):
        if getattr(self, "h", None):
            load().tt_cross_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self):
        self.status = check(load().tt_cross_run(self.h))
        return self.status

    def run_async(self, stream=None):
        """Start the run without waiting (tt_cross_run_async); stream: a torch
        stream or a raw hipStream_t (None: the handle's)."""
        s = None if stream is None else C.c_void_p(getattr(stream, "cuda_stream", stream))
        check(load().tt_cross_run_async(self.h, s))

    def query(self):
        """Advance the run in flight without blocking (tt_cross_query): 0
        while it runs, 1 when none is in flight."""
        return check(load().tt_cross_query(self.h))

    def wait(self):
        """Finish the run in flight and return its status (tt_cross_wait)."""
        self.status = check(load().tt_cross_wait(self.h))
        return self.status

    def set_rank_caps(self, caps):
        """Prescribed ranks: unfolding k stops at min(r_max, caps[k-1]) pivots
        (tt_cross_set_rank_caps); None clears them."""
        if caps is None:
            check(load().tt_cross_set_rank_caps(self.h, None))
        else:
            c = _i32(caps)
            check(load().tt_cross_set_rank_caps(self.h, c.ctypes.data_as(C.POINTER(C.c_int32))))

    def autotune(self, reps=3):
        """Time complete solves under every candidate tile shape (tt_autotune)
        and record the fastest for this problem's class; returns
        (tile_rows, tile_cols, ms), 0/0 meaning the library's default shape."""
        tr, tc, ms = C.c_int32(), C.c_int32(), C.c_double()
        check(load().tt_autotune(self.h, reps, C.byref(tr), C.byref(tc), C.byref(ms)))
        return tr.value, tc.value, ms.value

    def tiles(self):
        """(rows, cols) tile shape of each unfolding in the last run."""
        r = np.zeros(self.d - 1, dtype=np.int32)
        c = np.zeros(self.d - 1, dtype=np.int32)
        check(load().tt_cross_get_tiles(self.h, r.ctypes.data_as(C.POINTER(C.c_int32)),
                                        c.ctypes.data_as(C.POINTER(C.c_int32))))
        return list(zip(r.tolist(), c.tolist()))

    def ranks(self):
        r = np.zeros(self.d + 1, dtype=np.int32)
        check(load().tt_cross_get_ranks(self.h, r.ctypes.data_as(C.POINTER(C.c_int32))))
        return r

    def cores_flat(self):
        m = check(load().tt_cross_get_cores(self.h, None, 0, 0))
        out = np.zeros(m, dtype=np.float64)
        check(load().tt_cross_get_cores(self.h, out.ctypes.data_as(C.c_void_p), m, 0))
        return out

    def cores(self):
        flat, r = self.cores_flat(), self.ranks()
        res, off = [], 0
        for k in range(self.d):
            sz = int(r[k]) * int(self.n[k]) * int(r[k + 1])
            res.append(flat[off:off + sz].reshape(int(r[k]), int(self.n[k]), int(r[k + 1])))
            off += sz
        return res

    def pivots(self, k):
        rk = int(self.ranks()[k])
        rows = np.zeros((rk, k), dtype=np.int32)
        cols = np.zeros((rk, self.d - k), dtype=np.int32)
        check(load().tt_cross_get_pivots(self.h, k, rows.ctypes.data_as(C.c_void_p),
                                         cols.ctypes.data_as(C.c_void_p)))
        return rows, cols

    def history(self, k):
        cap = 4096
        out = np.zeros(cap, dtype=np.float64)
        m = check(load().tt_cross_get_history(self.h, k, out.ctypes.data_as(C.c_void_p), cap))
        return out[:min(m, cap)].copy()

    def stats(self):
        s = Stats()
        check(load().tt_cross_get_stats(self.h, C.byref(s)))
        return _stats_dict(s, self.d)

    def tt_eval(self, idx):
        """TT values at multi-indices: numpy (m, d) int32 on the host, or an
        int32 torch CUDA tensor (result on the device)."""
        if hasattr(idx, "is_cuda") and idx.is_cuda:
            import torch
            idx = idx.contiguous()
            out = torch.empty(idx.shape[0], dtype=torch.float64, device=idx.device)
            check(load().tt_eval(self.h, idx.shape[0], C.c_void_p(idx.data_ptr()), C.c_void_p(out.data_ptr()), 1))
            return out
        idx = _i32(np.atleast_2d(idx))
        out = np.zeros(idx.shape[0], dtype=np.float64)
        check(load().tt_eval(self.h, idx.shape[0], idx.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p), 0))
        return out

    def sampled_error(self, R=1_000_000, seed=1):
        e = C.c_double()
        check(load().tt_cross_sampled_error(self.h, R, C.c_uint64(seed), C.byref(e)))
        return e.value

    def sampled_error_noalloc(self, R=65536, seed=1):
        """The same error from the library's static scratch array
        (tt_cross_sampled_error_noalloc): no device allocation, R <= 65536."""
        e = C.c_double()
        check(load().tt_cross_sampled_error_noalloc(self.h, R, C.c_uint64(seed), C.byref(e)))
        return e.value


def batch_run(problems, stream=None):
    """Solve several TTCross problems together on one GPU (tt_batch_run).

    Each problem ends exactly as its own run() would end; the per-problem
    status is returned as a list (also in each problem's stats())."""
    problems = list(problems)
    arr = (C.c_void_p * len(problems))(*[p.h for p in problems])
    s = None if stream is None else C.c_void_p(getattr(stream, "cuda_stream", stream))
    L = load()
    check(L.tt_batch_run(arr, len(problems), s))
    # the statuses only, in one call (a stats() dictionary, or even a stats
    # call, per problem would cost more host time than a small batch's GPU
    # work)
    sts = (C.c_int32 * len(problems))()
    check(L.tt_batch_statuses(arr, len(problems), sts))
    out = list(sts)
    for p, v in zip(problems, out):
        p.status = v
    return out


def batch_autotune(problems, reps=2, per_class=16, stream=None):
    """Tune tile shapes per problem class on batched solves (tt_batch_autotune);
    returns the number of classes tuned."""
    problems = list(problems)
    arr = (C.c_void_p * len(problems))(*[p.h for p in problems])
    s = None if stream is None else C.c_void_p(getattr(stream, "cuda_stream", stream))
    return check(load().tt_batch_autotune(arr, len(problems), reps, per_class, s))


def tile_table():
    """The tuned tile shapes, one dict per problem class (tt_tile_table)."""
    L = load()
    n = L.tt_tile_table(None, 0)
    W = _lib.TILE_ROW_WORDS
    buf = np.zeros((max(n, 1), W), dtype=np.int32)
    n = L.tt_tile_table(buf.ctypes.data_as(C.c_void_p), n)
    D = _lib.TT_MAX_D
    out = []
    for row in buf[:n]:
        d = int(row[0])
        out.append({"d": d, "fp32": int(row[1]), "hilbert": int(row[2]), "r_max": int(row[3]),
                    "n": [int(x) for x in row[4:4 + d]], "grid": [int(x) for x in row[4 + D:4 + D + d]],
                    "tile_rows": int(row[4 + 2 * D]), "tile_cols": int(row[5 + 2 * D])})
    return out


def tile_table_clear():
    load().tt_tile_table_clear()


class Server:
    """Continuous-batching server (tt_server_*): submit requests at any time,
    wait for them, read their stats and cores."""

    def __init__(self, hbm_budget, max_slots=256, r_max=32, grid=2, precision=_lib.PREC_AUTO,
                 n_samples=16384, lookahead=2, verify=-1):
        L = load()
        o = default_options()
        o.r_max = r_max
        o.precision = precision
        o.n_samples = n_samples
        o.lookahead = lookahead
        o.verify = verify
        for j in range(_lib.TT_MAX_D):
            o.grid[j] = int(grid)
        self.h = L.tt_server_create(int(hbm_budget), int(max_slots), C.byref(o))
        if not self.h:
            raise _lib.TTError(_lib.EDEVICE, _lib.last_error())
        self._d = {}

    def submit(self, n, eps, fn_id, params=None, seed=0):
        n = _i32(n)
        pp, npar, _keep = _params_ptr(params)
        t = C.c_uint64()
        check(load().tt_server_submit(self.h, n.size, n.ctypes.data_as(C.POINTER(C.c_int32)), float(eps), fn_id,
                                      pp, npar, seed, C.byref(t)))
        self._d[t.value] = int(n.size)
        return t.value

    def poll(self, ticket):
        return check(load().tt_server_poll(self.h, ticket))

    def wait(self, ticket):
        """(status, latency in seconds from submission to completion)."""
        lat = C.c_double()
        st = check(load().tt_server_wait(self.h, ticket, C.byref(lat)))
        return st, lat.value

    def result(self, ticket):
        s = Stats()
        m = check(load().tt_server_result(self.h, ticket, C.byref(s), None, 0))
        cores = np.zeros(m, dtype=np.float64)
        check(load().tt_server_result(self.h, ticket, None, cores.ctypes.data_as(C.c_void_p), m))
        return _stats_dict(s, self._d.get(ticket, s.d)), cores

    def release(self, ticket):
        check(load().tt_server_release(self.h, ticket))
        self._d.pop(ticket, None)

    def stats(self):
        s = _lib.ServerStats()
        check(load().tt_server_get_stats(self.h, C.byref(s)))
        return {name: getattr(s, name) for name, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            load().tt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
