"""Served solves (tt_server_*): a request solved among others, admitted while
others run, must end bit for bit where its own single solve ends; the
server pools device buffers and keeps within its HBM budget."""
import time

import numpy as np
import pytest

from paper_2407_11290_amd import EINVAL, ENOMEM, FN_BIMAXWELL, FN_HILBERT, TTError
from paper_2407_11290_amd.api import Server, TTCross

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _bimax(seed):
    rng = np.random.default_rng(seed)
    p = []
    for _ in range(2):
        p += [rng.uniform(0.5, 2.0), *rng.uniform(-2.0, 2.0, 3), rng.uniform(0.5, 2.0)]
    return list(p) + [8.0]


def _requests():
    out = []
    shapes = [(3, 16), (3, 24), (4, 16), (4, 12), (5, 10), (3, 32)]
    for i in range(24):
        d, n = shapes[i % len(shapes)]
        eps = 1e-4 if i % 3 == 0 else 1e-8
        if i % 2 == 0:
            fn, params = FN_HILBERT, [0.25 * (i % 7)]
        else:
            fn, params = FN_BIMAXWELL, _bimax(i)
        out.append(dict(n=[n] * d, eps=eps, fn=fn, params=params, seed=1000 + i))
    return out


def _single(r):
    g = TTCross(r["n"], r["eps"], r["fn"], r["params"], seed=r["seed"], r_max=32, grid=[2] * len(r["n"]))
    st = g.run()
    return st, g.stats(), g.cores_flat()


def test_served_requests_equal_single_solves():
    reqs = _requests()
    srv = Server(8 << 30, max_slots=8)
    tickets = []
    # three waves: later requests join the rounds of earlier ones
    for w in range(3):
        for r in reqs[w * 8:(w + 1) * 8]:
            tickets.append(srv.submit(r["n"], r["eps"], r["fn"], r["params"], seed=r["seed"]))
        time.sleep(0.002)
    _say("submitted", len(tickets))
    for t, r in zip(tickets, reqs):
        st, lat = srv.wait(t)
        assert st >= 0 and lat > 0
        s, cores = srv.result(t)
        _say("check", r["n"], r["fn"], r["eps"], r["seed"])
        st1, s1, c1 = _single(r)
        assert s["status"] == st1
        for key in ("ranks", "sweeps", "pivoted", "evaluated", "rms", "tau", "precision_used"):
            assert s[key] == s1[key], (key, s[key], s1[key])
        assert np.array_equal(cores.view(np.uint64), c1.view(np.uint64))
        srv.release(t)
    info = srv.stats()
    assert info["completed"] == len(reqs) and info["queued"] == 0 and info["running"] == 0
    srv.close()


def test_server_pools_device_buffers():
    reqs = _requests()[:6]
    srv = Server(8 << 30, max_slots=4)
    for rnd in range(2):
        ts = [srv.submit(r["n"], r["eps"], r["fn"], r["params"], seed=r["seed"]) for r in reqs]
        for t in ts:
            assert srv.wait(t)[0] >= 0
            srv.release(t)
        if rnd == 0:
            first = srv.stats()["allocations"]
    assert srv.stats()["allocations"] == first
    srv.close()


def test_server_budget_limits():
    small = dict(n=[16] * 3, eps=1e-8, fn=FN_HILBERT, params=[1.0])
    other = dict(n=[12] * 4, eps=1e-8, fn=FN_HILBERT, params=[2.0])
    # a budget that holds one problem object at a time: shapes are evicted in turn
    probe = Server(8 << 30, max_slots=2)
    t = probe.submit(other["n"], other["eps"], other["fn"], other["params"])
    probe.wait(t)
    need = probe.stats()["pool_bytes"]
    probe.close()
    srv = Server(need + 4096, max_slots=2)
    ts = []
    for i in range(4):
        r = small if i % 2 == 0 else other
        ts.append(srv.submit(r["n"], r["eps"], r["fn"], r["params"], seed=i))
    for t in ts:
        assert srv.wait(t)[0] >= 0
    assert srv.stats()["pool_bytes"] <= need + 4096
    # a request larger than the whole budget fails, and the server goes on
    t = srv.submit([64] * 4, 1e-8, FN_HILBERT, [1.0])
    with pytest.raises(TTError) as e:
        srv.wait(t)
    assert e.value.code == ENOMEM
    t = srv.submit(small["n"], small["eps"], small["fn"], small["params"])
    assert srv.wait(t)[0] >= 0
    with pytest.raises(TTError) as e:
        srv.poll(123456)
    assert e.value.code == EINVAL
    srv.close()


def test_server_escalates_like_a_single_solve():
    """The mixed batch's problem 190 misses eps with FP32 sweeps; served, it is
    re-queued with FP64 sweeps and ends as its single solve does."""
    from paper_2407_11290_amd.workloads import batch_mix
    p = batch_mix()[190]
    srv = Server(16 << 30, max_slots=4, r_max=64, grid=2)
    t = srv.submit(p.n, p.eps, p.fn_id, p.params, seed=p.seed)
    assert srv.wait(t)[0] == 0
    s, cores = srv.result(t)
    g = TTCross(p.n, p.eps, p.fn_id, p.params, seed=p.seed, r_max=64, grid=p.grid)
    g.run()
    s1 = g.stats()
    assert s["escalated"] == 1 == s1["escalated"]
    for key in ("ranks", "sweeps", "pivoted", "precision_used", "sampled_err"):
        assert s[key] == s1[key], key
    assert np.array_equal(cores.view(np.uint64), g.cores_flat().view(np.uint64))
    srv.close()



def test_pooled_problem_switches_functions():
    """One pooled problem object serves, in turn, a Hilbert request and
    bi-Maxwellians with different parameters (whose per-mode tables are
    uploaded into the object's buffers); each result equals its single solve."""
    n = [16] * 4
    seq = [(FN_HILBERT, [0.5]), (FN_BIMAXWELL, _bimax(3)), (FN_HILBERT, [1.25]), (FN_BIMAXWELL, _bimax(4)),
           (FN_BIMAXWELL, _bimax(3))]
    srv = Server(8 << 30, max_slots=1)
    for i, (fn, params) in enumerate(seq):
        r = dict(n=n, eps=1e-8, fn=fn, params=params, seed=70 + i)
        _say("switch", i, fn)
        t = srv.submit(r["n"], r["eps"], r["fn"], r["params"], seed=r["seed"])
        st, _ = srv.wait(t)
        assert st >= 0
        s, cores = srv.result(t)
        st1, s1, c1 = _single(r)
        assert s["status"] == st1 and s["ranks"] == s1["ranks"] and s["pivoted"] == s1["pivoted"]
        assert np.array_equal(cores.view(np.uint64), c1.view(np.uint64))
        srv.release(t)
    assert srv.stats()["allocations"] == 1
    srv.close()
