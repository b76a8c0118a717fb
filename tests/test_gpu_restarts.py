"""Restarts after false convergence on the GPU (tt_options.restarts; not in
the paper) against the oracle's restarts: the same point list, pivots and
cores where the entries are bitwise the oracle's (separable sums), the same
outcome where they differ by the device exponential's rounding (the
interleaved-order Maxwellian)."""
import numpy as np
import pytest

from oracle import Oracle, fn_eval as orc_fn_eval
from paper_2407_11290_amd import FN_HILBERT, FN_MAXWELL_IL, FN_SEPSUM, PREC_FP64, TTError
from paper_2407_11290_amd.api import TTCross, fn_eval as gpu_fn_eval

pytestmark = pytest.mark.gpu

R_CHECK = 4096
OK, WARN_SAMPLED_ERR = 0, 2


def _say(*a):
    print("[case]", *a, flush=True)


def _two_blocks(n, A=1.0, B=2.0):
    params = [2.0]
    for c, low in ((A, True), (B, False)):
        for j, m in enumerate(n):
            v = [1.0 if ((i < m // 2) == low) else 0.0 for i in range(m)]
            params += [c * x for x in v] if j == 0 else v
    return np.array(params)


def _assert_same_pivots(g, o):
    assert list(g.ranks()) == list(o.ranks())
    for k in range(1, g.d):
        gr, gc = g.pivots(k)
        orows, ocols, *_ = o.pivots(k)
        assert np.array_equal(gr, orows), (k, gr, orows)
        assert np.array_equal(gc, ocols), (k, gc, ocols)


def _pair(n, eps, fn_id, params, seed, restarts):
    _say("restarts", fn_id, n, eps, seed, restarts)
    g = TTCross(n, eps, fn_id, params, seed=seed, precision=PREC_FP64, verify=R_CHECK, restarts=restarts)
    o = Oracle(n, eps, fn_id, params, seed=seed, restarts=restarts, restart_R=R_CHECK)
    return g, g.run(), o, o.run()


def test_interleaved_maxwellian_values():
    n = [8, 16, 9, 12, 7, 10]
    rng = np.random.default_rng(3)
    idx = np.stack([rng.integers(0, m, 20000) for m in n], axis=1).astype(np.int32)
    a = gpu_fn_eval(FN_MAXWELL_IL, n, idx)
    b = orc_fn_eval(FN_MAXWELL_IL, n, idx)
    # per-index factors from the FP64 table, the exponential on the device
    assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)) < 1e-15


@pytest.mark.parametrize("n", [[16, 16, 16], [12, 10, 14, 8]])
def test_two_block_tensor_restart_is_the_oracles(n):
    g, gs, o, os_ = _pair(n, 1e-8, FN_SEPSUM, _two_blocks(n), 0, 3)
    st, info = g.stats(), o.restart_info()
    assert gs == os_ == OK
    assert st["restarts_used"] == info["used"] == 1 and st["restart_cause"] == info["cause"] == 0
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())
    assert st["sampled_err"] <= 1e-8 and info["err"] <= 1e-8
    # the same problem through the stepwise run
    a = TTCross(n, 1e-8, FN_SEPSUM, _two_blocks(n), seed=0, precision=PREC_FP64, verify=R_CHECK, restarts=3)
    a.run_async()
    assert a.wait() == OK
    assert np.array_equal(a.cores_flat(), g.cores_flat())


def _framed_two_blocks(n, A=1.0, B=2.0):
    d = len(n)
    params = [2.0]
    for c, low in ((A, True), (B, False)):
        for j, m in enumerate(n):
            if j == 0:
                v = [c * (1.0 + 0.1 * i) for i in range(m)]
            elif j == d - 1:
                v = [2.0 - 0.1 * i for i in range(m)]
            else:
                v = [1.0 if ((i < m // 2) == low) else 0.0 for i in range(m)]
            params += v
    return np.array(params)


@pytest.mark.parametrize("n", [[6, 8, 8, 8, 8, 5], [5, 6, 7, 6, 4]])
def test_trimmed_restart_point_is_the_oracles(n):
    """The restart point is trimmed to i0's end indices (zero residual in the
    rank-1 end unfoldings): same point, pivots and cores as the oracle."""
    g, gs, o, os_ = _pair(n, 1e-8, FN_SEPSUM, _framed_two_blocks(n), 0, 3)
    st, info = g.stats(), o.restart_info()
    assert gs == os_ == OK and st["restarts_used"] == info["used"] == 1
    _assert_same_pivots(g, o)
    assert np.array_equal(g.cores_flat(), o.cores_flat())


@pytest.mark.parametrize("seed", [0, 2])
def test_interleaved_maxwellian_reaches_eps_like_the_oracle(seed):
    """Same outcome as the oracle: status, restarts, ranks, and the error on
    an independent stream.  The pivots themselves may differ: the tensor is
    symmetric under v -> -v, so many residuals tie exactly in exact
    arithmetic and the device exponential's rounding breaks those ties
    differently (as in the plain Maxwellian parity tests)."""
    n, eps = [16] * 6, 1e-6
    g, gs, o, os_ = _pair(n, eps, FN_MAXWELL_IL, None, seed, 8)
    st, info = g.stats(), o.restart_info()
    _say("gpu", gs, st["restarts_used"], st["sampled_err"], list(g.ranks()), "oracle", os_, info["used"],
         info["err"], list(o.ranks()))
    assert gs == os_ == OK
    assert st["restarts_used"] == info["used"] and st["restart_cause"] == 0
    assert list(g.ranks()) == list(o.ranks())
    assert st["sampled_err"] <= eps
    assert g.sampled_error(20000, seed=seed + 7) <= 3 * eps


def test_restarts_used_up_is_reported():
    n, eps = [16] * 6, 1e-6
    g, gs, o, os_ = _pair(n, eps, FN_MAXWELL_IL, None, 0, 1)
    st, info = g.stats(), o.restart_info()
    assert gs == os_ == WARN_SAMPLED_ERR
    assert st["restarts_used"] == info["used"] == 1 and st["restart_cause"] == info["cause"] == 1
    assert st["sampled_err"] > eps


def test_runs_that_meet_eps_are_untouched():
    n, eps = [9, 8, 10, 7], 1e-9
    a = TTCross(n, eps, FN_HILBERT, seed=1, precision=PREC_FP64, verify=R_CHECK)
    b = TTCross(n, eps, FN_HILBERT, seed=1, precision=PREC_FP64, verify=R_CHECK, restarts=2)
    assert a.run() == b.run() == OK
    assert b.stats()["restarts_used"] == 0
    assert np.array_equal(a.cores_flat(), b.cores_flat())


def test_restart_options_are_checked():
    with pytest.raises(TTError):
        TTCross([8, 8, 8], 1e-8, FN_HILBERT, restarts=9)
    with pytest.raises(TTError):
        TTCross([8, 8, 8], 1e-8, FN_HILBERT, restarts=1, verify=0)
