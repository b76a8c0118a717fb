"""GPU parity: the HIP path against the FP64 CPU oracle on the same seeded inputs.

FP64 sweeps must reproduce the oracle's pivot index sets bit for bit, and the
cores (same FP64 operations in the same order) too; reconstructed entries must
agree within a relative 1e-12.  FP32 sweeps are compared by error against the
FP64 oracle, within 1e-5 relative.
"""
import itertools

import numpy as np
import pytest

from oracle import Oracle, fn_eval as orc_fn_eval
from paper_2407_11290_amd import (FN_BIMAXWELL, FN_HILBERT, FN_MAXWELL, FN_MAXWELL_2D2V, FN_MAXWELL_3D3V,
                                  FN_SEPSUM, NOT_CONVERGED, PREC_FP32, PREC_FP64)
from paper_2407_11290_amd.api import TTCross, fn_eval as gpu_fn_eval, fn_eval_last_kernel_ms

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _sepsum_params(n, r, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([[float(r)], 0.5 + rng.random(r * int(np.sum(n)))])


def _bimax_params(seed):
    rng = np.random.default_rng(seed)
    p = []
    for _ in range(2):
        p += [rng.uniform(0.5, 2.0), *rng.uniform(-2.0, 2.0, 3), rng.uniform(0.5, 2.0)]
    return np.array(p + [8.0])


def _solve_both(n, eps, fn_id, params=None, seed=0, r_max=64, **kw):
    _say("n", list(n), "eps", eps, "fn", fn_id, "seed", seed, kw)
    g = TTCross(n, eps, fn_id, params, seed=seed, r_max=r_max, **kw)
    gs = g.run()
    o = Oracle(n, eps, fn_id, params, seed=seed, r_max=r_max)
    os_ = o.run()
    return g, gs, o, os_


def _assert_same_pivots(g, o):
    assert list(g.ranks()) == list(o.ranks())
    for k in range(1, g.d):
        gr, gc = g.pivots(k)
        orows, ocols, *_ = o.pivots(k)
        assert np.array_equal(gr, orows), (k, gr, orows)
        assert np.array_equal(gc, ocols), (k, gc, ocols)


# --------------------------------------------------------------------------
# generating functions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("fn_id,n,params,exact", [
    (FN_HILBERT, [32, 32, 32], None, True),
    (FN_HILBERT, [64] * 6, None, True),
    (FN_HILBERT, [7, 9, 5, 11], [2.37], True),
    (FN_SEPSUM, [5, 6, 7], "sep", True),
    (FN_MAXWELL, [16] * 6, None, False),
    (FN_BIMAXWELL, [4, 16, 16, 16], "bimax", False),
    (FN_MAXWELL_2D2V, [20, 10, 20, 10], None, False),
    (FN_MAXWELL_3D3V, [8, 4, 8, 4, 8, 4], None, False),
])
def test_fn_values(fn_id, n, params, exact):
    if isinstance(params, str):
        params = _sepsum_params(n, 3, 1) if params == "sep" else _bimax_params(2)
    rng = np.random.default_rng(5)
    idx = np.stack([rng.integers(0, m, 20000) for m in n], axis=1).astype(np.int32)
    _say("fn values", fn_id, n)
    a = gpu_fn_eval(fn_id, n, idx, params)
    b = orc_fn_eval(fn_id, n, idx, params)
    if exact:
        assert np.array_equal(a, b)
    else:
        # the Maxwellians' per-index factors come from a table built in FP64 by
        # the formula's own operations, so entries differ from the oracle's
        # only by the device exponential's rounding: a few ulps
        rel = np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))
        _say("fn values max relative difference", rel)
        assert rel < 1e-15


@pytest.mark.parametrize("fn_id,n,params", [
    (FN_HILBERT, [64] * 6, None),
    (FN_HILBERT, [7, 9, 5, 11], [2.37]),
    (FN_SEPSUM, [5, 6, 7], "sep"),
    (FN_MAXWELL, [128] * 6, None),
    (FN_BIMAXWELL, [4, 16, 16, 16], "bimax"),
    (FN_MAXWELL_2D2V, [20, 10, 20, 10], None),
    (FN_MAXWELL_3D3V, [8, 4, 8, 4, 8, 4], None),
])
def test_fp32_fn_values_against_fp64_oracle(fn_id, n, params):
    """Entries in the FP32 arithmetic of FP32 sweeps: within a few FP32
    roundings of the FP64 oracle.  Entries far below the largest may lose
    relative accuracy (exp underflows to FP32 subnormals), so they are held
    to an absolute bound of the largest entry's scale."""
    if isinstance(params, str):
        params = _sepsum_params(n, 3, 1) if params == "sep" else _bimax_params(2)
    rng = np.random.default_rng(6)
    idx = np.stack([rng.integers(0, m, 50000) for m in n], axis=1).astype(np.int32)
    _say("fp32 fn values", fn_id, n)
    a = gpu_fn_eval(fn_id, n, idx, params, fp32=True)
    assert a.dtype == np.float32
    b = orc_fn_eval(fn_id, n, idx, params)
    err = np.abs(a.astype(np.float64) - b)
    scale = np.max(np.abs(b))
    assert np.max(err) <= 2e-6 * scale
    big = np.abs(b) >= 1e-3 * scale
    assert np.max(err[big] / np.abs(b[big])) <= 1e-5
    if fn_id == FN_HILBERT and params is None:
        # integer shift: one correctly rounded FP32 division of an exact integer
        assert np.max(err / np.abs(b)) <= 2.0 ** -24


# --------------------------------------------------------------------------
# FP64: bit-exact pivots and cores
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", list(range(10)))
def test_hilbert3d_n32_bit_exact(seed):
    """3D Hilbert tensor, n = 32, eps = 1e-10, FP64 (the 32768-entry case)."""
    g, gs, o, os_ = _solve_both([32, 32, 32], 1e-10, FN_HILBERT, seed=seed, precision=PREC_FP64)
    assert gs == os_ == 0
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())
    st, ost = g.stats(), o.stats()
    assert st["rms"] == ost["rms"] and st["tau"] == ost["tau"]
    assert st["sweeps"] == ost["sweeps"] and st["pivoted"] == ost["pivoted"]
    assert st["evaluated"] == ost["evaluated"]
    for k in (1, 2):
        assert np.array_equal(g.history(k), o.history(k))
    # every entry of the tensor: reconstruction and error
    idx = np.array(list(itertools.product(range(32), range(32), range(32))), dtype=np.int32)
    y = g.tt_eval(idx)
    assert np.array_equal(y, o.tt_eval(idx))
    x = orc_fn_eval(FN_HILBERT, [32, 32, 32], idx)
    assert np.linalg.norm(x - y) / np.linalg.norm(x) <= 1e-10


@pytest.mark.parametrize("n,grid,tiles", [
    ([13, 17, 11, 19], [1, 1, 1, 1], (8, 8)),
    ([13, 17, 11, 19], [2, 3, 1, 2], (4, 4)),
    ([13, 17, 11, 19], [1, 1, 1, 1], (32, 64)),
    ([5, 40, 3, 7, 9], [1, 4, 1, 1, 2], (16, 16)),
    ([2, 2, 2, 2, 2, 2, 2, 2], [1] * 8, (0, 0)),
    # tiles taller than 64 rows: stored tiles in several 64-row chunks, the last ragged
    ([13, 17, 11, 19], [1, 1, 1, 1], (128, 32)),
    ([13, 17, 11, 19], [1, 1, 1, 1], (100, 8)),
    ([5, 40, 3, 7, 9], [1, 1, 1, 1, 1], (192, 16)),
])
def test_ragged_tiles_and_grids_bit_exact(n, grid, tiles):
    """Several tiles per superblock with ragged tails, and uneven subtensor blocks."""
    g, gs, o, os_ = _solve_both(n, 1e-9, FN_HILBERT, seed=3, precision=PREC_FP64, grid=grid,
                                tile_rows=tiles[0], tile_cols=tiles[1])
    assert gs == os_
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_hilbert6d_n64_grid2_bit_exact(seed):
    """6D Hilbert tensor, n = 64, 2^6 subtensor blocks, eps = 1e-8, FP64."""
    n = [64] * 6
    g, gs, o, os_ = _solve_both(n, 1e-8, FN_HILBERT, seed=seed, precision=PREC_FP64, grid=[2] * 6)
    assert gs == os_ == 0
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())
    st, ost = g.stats(), o.stats()
    assert st["pivoted"] == ost["pivoted"] and st["evaluated"] == ost["evaluated"]
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 64, (20000, 6)).astype(np.int32)
    assert np.max(np.abs(g.tt_eval(idx) - o.tt_eval(idx))) <= 1e-12 * np.max(np.abs(orc_fn_eval(FN_HILBERT, n, idx)))
    assert g.sampled_error(1_000_000, seed + 1) <= 1e-8


def test_block_grid_invariance():
    """Sec. 3.2.1: the global pivot is the best of the local pivots, so greedy
    pivots do not depend on the subtensor grid."""
    n = [24, 24, 24, 24]
    ref = None
    for grid in ([1, 1, 1, 1], [2, 2, 2, 2], [1, 3, 2, 1], [4, 1, 1, 4], [3, 3, 3, 3]):
        _say("grid", grid)
        g = TTCross(n, 1e-9, FN_HILBERT, seed=1, precision=PREC_FP64, grid=grid)
        g.run()
        piv = [g.pivots(k) for k in range(1, 4)]
        if ref is None:
            ref = piv
        else:
            for (a, b), (c, e) in zip(piv, ref):
                assert np.array_equal(a, c) and np.array_equal(b, e)


def test_sepsum_exact_recovery_bit_exact():
    n = [9, 10, 11, 8, 7]
    params = _sepsum_params(n, 4, 2)
    g, gs, o, os_ = _solve_both(n, 1e-12, FN_SEPSUM, params, seed=7, precision=PREC_FP64)
    _assert_same_pivots(g, o)
    assert (g.ranks()[1:-1] <= 4).all()
    assert np.array_equal(g.cores_flat(), o.cores_flat())


def test_bimaxwellian_rank_two():
    n = [8, 32, 32, 32]
    p = _bimax_params(3)
    g, gs, o, os_ = _solve_both(n, 1e-10, FN_BIMAXWELL, p, seed=1, precision=PREC_FP64)
    assert (g.ranks()[1:-1] <= 2).all()
    rng = np.random.default_rng(0)
    idx = np.stack([rng.integers(0, m, 5000) for m in n], axis=1).astype(np.int32)
    x = orc_fn_eval(FN_BIMAXWELL, n, idx, p)
    assert np.linalg.norm(g.tt_eval(idx) - x) / np.linalg.norm(x) < 1e-10


def test_rank_cap_and_d2_edge_cases():
    g, gs, o, os_ = _solve_both([16, 16, 16], 1e-14, FN_HILBERT, seed=0, r_max=4, precision=PREC_FP64)
    assert gs == os_ == NOT_CONVERGED
    _assert_same_pivots(g, o)
    # d = 2 (a matrix), a mode of size 1, and a tiny full-rank case
    for n in ([100, 100], [1, 30, 30], [3, 1, 4], [2, 3]):
        g, gs, o, os_ = _solve_both(n, 1e-12, FN_HILBERT, seed=2, precision=PREC_FP64)
        assert gs == os_
        _assert_same_pivots(g, o)
        assert np.array_equal(g.cores_flat(), o.cores_flat())


def test_eval_on_device_tensors():
    import torch
    g = TTCross([32, 32, 32], 1e-10, FN_HILBERT, seed=0, precision=PREC_FP64)
    g.run()
    idx = torch.randint(0, 32, (10000, 3), dtype=torch.int32, device="cuda")
    y = g.tt_eval(idx).cpu().numpy()
    assert np.array_equal(y, g.tt_eval(idx.cpu().numpy()))
    x = gpu_fn_eval(FN_HILBERT, [32, 32, 32], idx).cpu().numpy()
    assert np.array_equal(x, orc_fn_eval(FN_HILBERT, [32, 32, 32], idx.cpu().numpy()))
    # the kernel's own duration, from events attached to its dispatch
    ms = fn_eval_last_kernel_ms()
    assert 0.0 < ms < 1000.0


def test_fn_eval_tables_follow_the_function():
    """Bulk evaluation keeps the per-mode tables of recent functions on the
    device: a change of parameters, of function or of shape, and a return to
    an earlier one after more than four others, all give the oracle's values."""
    rng = np.random.default_rng(8)
    cases = []
    for i in range(6):
        n = [4, 16, 16, 16] if i % 2 == 0 else [3, 12, 12, 12]
        cases.append((FN_BIMAXWELL, n, _bimax_params(i)))
    cases += [(FN_MAXWELL, [16] * 6, [0.4, 0.2, 1.5, 6.0]), (FN_MAXWELL, [16] * 6, None),
              (FN_MAXWELL_2D2V, [20, 10, 20, 10], None)]
    cases += cases[:3]
    for fn_id, n, params in cases:
        idx = np.stack([rng.integers(0, m, 5000) for m in n], axis=1).astype(np.int32)
        _say("table", fn_id, n)
        a = gpu_fn_eval(fn_id, n, idx, params)
        b = orc_fn_eval(fn_id, n, idx, params)
        assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)) < 1e-13
        a32 = gpu_fn_eval(fn_id, n, idx, params, fp32=True)
        assert np.max(np.abs(a32.astype(np.float64) - b)) <= 2e-6 * np.max(np.abs(b))


# --------------------------------------------------------------------------
# FP32 sweeps with FP64 pivot check, stop test and cores
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_maxwellian6d_fp32_against_fp64_oracle(seed):
    """Single 3d3v Maxwellian, n = 128, eps = 1e-6: FP32 sweeps, FP64 check."""
    n = [128] * 6
    g, gs, o, os_ = _solve_both(n, 1e-6, FN_MAXWELL, seed=seed, precision=PREC_FP32, grid=[2] * 6)
    assert g.stats()["precision_used"] == PREC_FP32
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 128, (100000, 6)).astype(np.int32)
    yg, yo = g.tt_eval(idx), o.tt_eval(idx)
    x = orc_fn_eval(FN_MAXWELL, n, idx)
    # reconstructed entries within 1e-5 of the FP64 oracle's (relative to max |X|)
    assert np.max(np.abs(yg - yo)) <= 1e-5 * np.max(np.abs(x))
    assert g.sampled_error(1_000_000, 11) <= 1e-6


def test_hilbert_fp32_sweeps_meet_eps():
    n = [32] * 5
    g, gs, o, os_ = _solve_both(n, 1e-6, FN_HILBERT, seed=4, precision=PREC_FP32)
    assert g.sampled_error(200_000, 3) <= 1e-6
    rng = np.random.default_rng(1)
    idx = rng.integers(0, 32, (20000, 5)).astype(np.int32)
    x = orc_fn_eval(FN_HILBERT, n, idx)
    assert np.max(np.abs(g.tt_eval(idx) - o.tt_eval(idx))) <= 1e-5 * np.max(np.abs(x))


def o_status(o):
    from oracle.oracle import lib as orc_lib
    return orc_lib().orc_run(o.h)


@pytest.mark.parametrize("pivot", ["greedy", "rook"])
def test_degenerate_and_maximum_shapes(pivot):
    """A one-entry tensor, eps = 0 (the search runs until the residual is
    exactly zero or the rank cap), rank cap 1, the largest number of modes
    (16), and a matrix driven to the full rank cap of 64: same pivots, ranks,
    cores and status as the oracle, in greedy and in rook mode."""
    from paper_2407_11290_amd import PIVOT_ROOK
    cases = [
        ([1, 1, 1], 1e-8, 64, None),
        ([4, 5, 3], 0.0, 64, [2, 2, 1]),
        ([9, 7, 8], 1e-12, 1, [2, 1, 2]),
        ([2] * 16, 1e-10, 64, [2] * 16),
        ([200, 180], 0.0, 64, [2, 3]),
    ]
    for n, eps, r_max, grid in cases:
        _say("degenerate", pivot, n, eps, r_max, grid)
        kw = dict(seed=1, r_max=r_max, precision=PREC_FP64)
        if grid is not None:
            kw["grid"] = grid
        if pivot == "rook":
            g = TTCross(n, eps, FN_HILBERT, pivot=PIVOT_ROOK, **kw)
            o = Oracle(n, eps, FN_HILBERT, seed=1, r_max=r_max, pivot="rook", grid=grid)
        else:
            g = TTCross(n, eps, FN_HILBERT, **kw)
            o = Oracle(n, eps, FN_HILBERT, seed=1, r_max=r_max)
        from paper_2407_11290_amd import _lib
        gs = _lib.load().tt_cross_run(g.h)      # the status code, errors included
        os_ = o_status(o)
        assert gs == os_, (n, gs, os_)
        if gs < 0:
            # driven to rounding noise (eps = 0): both sides find the same
            # zero pivot-block residual in Alg. 4
            continue
        _assert_same_pivots(g, o)
        assert np.array_equal(g.cores_flat(), o.cores_flat())
        if n == [1, 1, 1]:
            assert list(g.ranks()) == [1, 1, 1, 1]
        if r_max == 1:
            assert max(g.ranks()) == 1


@pytest.mark.parametrize("pivot", ["greedy", "rook"])
def test_prescribed_ranks_match_the_oracle(pivot):
    """Per-unfolding rank caps with eps = 0 (the paper's fixed-rank runs):
    the GPU stops every unfolding at its cap with the oracle's pivots and
    cores, in greedy and rook mode."""
    from paper_2407_11290_amd import PIVOT_ROOK
    n, caps, grid = [12, 10, 9, 8], [5, 3, 7], [2, 1, 2, 2]
    kw = dict(seed=2, precision=PREC_FP64, grid=grid)
    if pivot == "rook":
        g = TTCross(n, 0.0, FN_HILBERT, pivot=PIVOT_ROOK, **kw)
        o = Oracle(n, 0.0, FN_HILBERT, seed=2, pivot="rook", grid=grid, rank_caps=caps)
    else:
        g = TTCross(n, 0.0, FN_HILBERT, **kw)
        o = Oracle(n, 0.0, FN_HILBERT, seed=2, rank_caps=caps)
    g.set_rank_caps(caps)
    _say("prescribed ranks", pivot, n, caps)
    assert g.run() == o.run() == NOT_CONVERGED
    assert list(g.ranks()) == [1, 5, 3, 7, 1]
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())


def test_paper_table6_hilbert3d_prescribed_ranks():
    """The paper's Table 6 tensor (3D Hilbert, n = 250) at its core ranks
    (1, 25, 25, 1): the sampled error over 1e6 entries is at most the printed
    subtensor error, 1.27e-6 (one-sided: the greedy full search finds a far
    smaller error than the paper's run)."""
    g = TTCross([250] * 3, 0.0, FN_HILBERT, seed=0, precision=PREC_FP64, grid=[2, 2, 2])
    g.set_rank_caps([25, 25])
    assert g.run() == NOT_CONVERGED
    assert list(g.ranks()) == [1, 25, 25, 1]
    assert g.sampled_error(1_000_000) <= 1.27e-6


def test_default_tall_tiles_bit_exact():
    """Block runs of 400 and more take 256-row tiles by default: the same
    pivots, status and cores as the oracle (rank cap 12 reached)."""
    n = [400, 410, 420]
    g, gs, o, os_ = _solve_both(n, 1e-7, FN_HILBERT, seed=1, r_max=12, precision=PREC_FP64)
    assert [t[0] for t in g.tiles()] == [256, 256]
    assert gs == os_ == NOT_CONVERGED
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())


@pytest.mark.parametrize("fn_id,n", [(FN_MAXWELL, [4096] * 6), (FN_MAXWELL_3D3V, [3000, 1500, 3000, 1500, 3000, 1500])])
def test_fn_values_with_tables_too_large_for_lds(fn_id, n):
    """Per-mode tables above the bulk evaluation's LDS limit are read from
    device memory; the values are the same as through LDS."""
    rng = np.random.default_rng(9)
    idx = np.stack([rng.integers(0, m, 20000) for m in n], axis=1).astype(np.int32)
    _say("large tables", fn_id, n)
    a = gpu_fn_eval(fn_id, n, idx)
    b = orc_fn_eval(fn_id, n, idx)
    assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)) < 1e-15
    a32 = gpu_fn_eval(fn_id, n, idx, fp32=True)
    assert np.max(np.abs(a32.astype(np.float64) - b)) <= 2e-6 * np.max(np.abs(b))


@pytest.mark.parametrize("name,n,eps,fn_id,sep_r,caps,grid", [
    # ranks 24 (T in 32 registers per row), general function
    ("sep24", [40, 36, 32], 1e-13, FN_SEPSUM, 24, None, [2, 2, 2]),
    # ranks 40 (64 registers per row), general function
    ("sep40", [48, 44, 42], 1e-13, FN_SEPSUM, 40, None, [2, 1, 2]),
    # the Hilbert kernel's entries from integer index sums, ranks 20 and 28
    ("hil_20_28", [120, 100, 80], 0.0, FN_HILBERT, 0, [20, 28], [2, 2, 2]),
])
def test_cores_above_rank_16_match_the_oracle(name, n, eps, fn_id, sep_r, caps, grid):
    """Above rank 16 the pivot rows' recursion of Alg. 4 runs once per
    unfolding and the fiber rows apply its recorded steps with their T in
    registers: the same pivots, status and cores as the oracle, bit for bit."""
    params = _sepsum_params(n, sep_r, 3) if sep_r else None
    _say("cores above rank 16", name, n, eps, caps, grid)
    g = TTCross(n, eps, fn_id, params, seed=1, grid=grid, precision=PREC_FP64)
    if caps:
        g.set_rank_caps(caps)
        o = Oracle(n, eps, fn_id, params, seed=1, rank_caps=caps)
    else:
        o = Oracle(n, eps, fn_id, params, seed=1)
    gs, os_ = g.run(), o.run()
    assert gs == os_, (gs, os_)
    assert max(g.ranks()) > 16
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())
