"""tt_cross_run_async / tt_cross_query / tt_cross_wait: the run of Sec. 1
started without waiting, advanced by polling, and finished; its results must
be bit for bit those of tt_cross_run (the same launches in the same order),
and the handle refuses other calls while the run is in flight."""
import time

import numpy as np
import pytest

from oracle import Oracle
from paper_2407_11290_amd import ESTATE, FN_BIMAXWELL, FN_HILBERT, PREC_FP64, TTError
from paper_2407_11290_amd.api import TTCross

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _same(a, b):
    assert list(a.ranks()) == list(b.ranks())
    for k in range(1, a.d):
        for x, y in zip(a.pivots(k), b.pivots(k)):
            assert np.array_equal(x, y), k
        assert np.array_equal(a.history(k), b.history(k)), k
    assert np.array_equal(a.cores_flat(), b.cores_flat())
    sa, sb = a.stats(), b.stats()
    for key in ("status", "sweeps", "evaluated", "pivoted", "precision_used", "escalated", "sampled_err", "rms",
                "tau"):
        assert sa[key] == sb[key], key


def _poll(h):
    zeros, t0 = 0, time.perf_counter()
    while h.query() == 0:
        zeros += 1
        assert time.perf_counter() - t0 < 60.0
    return zeros


@pytest.mark.parametrize("n,eps,grid", [([2000] * 3, 1e-8, [2, 2, 2]), ([64] * 6, 1e-8, [2] * 6)])
def test_async_run_polls_and_matches_the_blocking_run(n, eps, grid):
    _say("async", n, eps, grid)
    a = TTCross(n, eps, FN_HILBERT, seed=1, grid=grid, precision=PREC_FP64)
    b = TTCross(n, eps, FN_HILBERT, seed=1, grid=grid, precision=PREC_FP64)
    assert b.run() == 0
    a.run()                                          # allocate, so that the timed start only launches
    t0 = time.perf_counter()
    a.run_async()
    started = time.perf_counter() - t0
    zeros = _poll(a)
    st = a.wait()
    _say("start took", started * 1e3, "ms; polls while running", zeros, "device time", a.stats()["time_to_eps_s"])
    assert zeros > 0                                 # it returned before the run was over
    assert started < a.stats()["time_to_eps_s"]
    assert st == 0
    _same(a, b)
    # again on the same handle, waiting without polling
    a.run_async()
    assert a.wait() == 0
    _same(a, b)
    # and the oracle agrees on the pivots (bit-exact FP64 path)
    if n == [64] * 6:
        o = Oracle(n, eps, FN_HILBERT, seed=1)
        o.run()
        for k in range(1, a.d):
            assert np.array_equal(a.pivots(k)[0], o.pivots(k)[0])


def test_async_fp32_run_with_check_and_escalation_matches_the_blocking_run():
    """A problem whose FP32 sweeps miss eps = 1e-6 (the precision policy then
    redoes it with FP64 sweeps): the escalation happens inside the polled
    run, and status, error and flags equal those of tt_cross_run."""
    n, eps = [128] * 6, 1e-6
    _say("async escalation", n)
    a = TTCross(n, eps, FN_HILBERT, seed=0, grid=[2] * 6)
    b = TTCross(n, eps, FN_HILBERT, seed=0, grid=[2] * 6)
    sb = b.run()
    a.run_async()
    _poll(a)
    assert a.wait() == sb
    _same(a, b)
    _say("escalated", a.stats()["escalated"], "sampled error", a.stats()["sampled_err"])
    # a bi-Maxwellian that FP32 sweeps do solve: checked, not escalated
    p = [0.9, 0.5, -1.0, 0.3, 0.7, 1.4, -0.2, 1.1, -1.5, 1.2, 8.0]
    c = TTCross([4, 64, 64, 64], eps, FN_BIMAXWELL, p, seed=3, grid=[2] * 4)
    e = TTCross([4, 64, 64, 64], eps, FN_BIMAXWELL, p, seed=3, grid=[2] * 4)
    e.run()
    c.run_async()
    assert c.wait() == e.stats()["status"]
    _same(c, e)
    assert c.stats()["sampled_err"] >= 0.0 and c.stats()["escalated"] == 0


def test_async_run_on_a_torch_stream():
    import torch
    s = torch.cuda.Stream()
    n = [32, 32, 32]
    a = TTCross(n, 1e-10, FN_HILBERT, seed=0, precision=PREC_FP64)
    b = TTCross(n, 1e-10, FN_HILBERT, seed=0, precision=PREC_FP64)
    b.run()
    a.run_async(s)
    assert a.wait() == 0
    _same(a, b)
    # the handle kept the stream: a blocking run there too
    assert a.run() == 0
    _same(a, b)


def test_calls_are_refused_while_a_run_is_in_flight():
    n = [2000] * 3
    a = TTCross(n, 1e-8, FN_HILBERT, seed=2, grid=[2, 2, 2], precision=PREC_FP64)
    a.run()
    a.run_async()
    refused = 0
    for call in (a.ranks, a.cores_flat, a.stats, lambda: a.pivots(1), a.run, lambda: a.set_rank_caps([3, 3]),
                 a.run_async):
        try:
            call()
        except TTError as e:
            assert e.code == ESTATE
            refused += 1
    assert a.wait() == 0
    assert refused == 7
    assert a.query() == 1                            # nothing in flight
    a.ranks()


def test_destroy_with_a_run_in_flight_finishes_it_first():
    a = TTCross([1000] * 3, 1e-8, FN_HILBERT, seed=0, grid=[2, 2, 2], precision=PREC_FP64)
    a.run()
    a.run_async()
    a.close()
    b = TTCross([64] * 3, 1e-8, FN_HILBERT, seed=0, precision=PREC_FP64)
    assert b.run() == 0


def test_wait_without_a_run_is_refused():
    a = TTCross([8, 8, 8], 1e-8, FN_HILBERT)
    with pytest.raises(TTError) as e:
        a.wait()
    assert e.value.code == ESTATE
    assert a.query() == 1
