"""Batched solves (tt_batch_run): every problem of a batch must end exactly
where its own single solve ends -- ranks, pivots, history, counts and cores
bit for bit -- and FP64 problems must match the FP64 oracle's pivots."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2407_11290_amd import FN_BIMAXWELL, FN_HILBERT, PREC_FP32, PREC_FP64
from paper_2407_11290_amd.api import TTCross, batch_run
from paper_2407_11290_amd.workloads import batch_mix

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _make(spec, **kw):
    return TTCross(spec["n"], spec["eps"], spec["fn"], spec.get("params"), seed=spec["seed"],
                   grid=spec.get("grid"), **kw)


def _snapshot(g):
    st = g.stats()
    piv = [g.pivots(k) for k in range(1, g.d)]
    hist = [g.history(k) for k in range(1, g.d)]
    return {
        "status": st["status"], "ranks": list(g.ranks()), "sweeps": st["sweeps"],
        "pivoted": st["pivoted"], "evaluated": st["evaluated"], "rms": st["rms"], "tau": st["tau"],
        "piv": piv, "hist": hist, "cores": g.cores_flat(), "prec": st["precision_used"],
    }


def _assert_same(a, b, tag):
    for key in ("status", "ranks", "sweeps", "pivoted", "evaluated", "rms", "tau", "prec"):
        assert a[key] == b[key], (tag, key, a[key], b[key])
    for (ra, ca), (rb, cb) in zip(a["piv"], b["piv"]):
        assert np.array_equal(ra, rb) and np.array_equal(ca, cb), tag
    for ha, hb in zip(a["hist"], b["hist"]):
        assert np.array_equal(ha, hb), tag
    assert a["cores"].shape == b["cores"].shape, tag
    assert np.array_equal(a["cores"].view(np.uint64), b["cores"].view(np.uint64)), tag


def _bimax(seed):
    rng = np.random.default_rng(seed)
    p = []
    for _ in range(2):
        p += [rng.uniform(0.5, 2.0), *rng.uniform(-2.0, 2.0, 3), rng.uniform(0.5, 2.0)]
    return list(p) + [8.0]


def _mixed_specs():
    specs = []
    for i, (d, n) in enumerate([(3, 16), (3, 32), (4, 16), (4, 20), (5, 16), (3, 33), (6, 8), (2, 40)]):
        specs.append({"n": [n] * d, "eps": 1e-9, "fn": FN_HILBERT, "params": [1.0 + 0.25 * i], "seed": i,
                      "grid": [1 + (i % 3)] * d, "precision": PREC_FP64})
    for i, (d, n) in enumerate([(3, 16), (4, 24), (5, 16), (6, 12)]):
        specs.append({"n": [n] * d, "eps": 1e-10, "fn": FN_BIMAXWELL, "params": _bimax(i), "seed": 100 + i,
                      "grid": [2] * d, "precision": PREC_FP64})
    for i, (d, n) in enumerate([(3, 32), (4, 16), (5, 24)]):
        specs.append({"n": [n] * d, "eps": 1e-6, "fn": FN_HILBERT, "params": [0.5 * i], "seed": 200 + i,
                      "grid": [2] * d, "precision": PREC_FP32})
    return specs


def test_mixed_batch_equals_single_solves():
    specs = _mixed_specs()
    singles = []
    for s in specs:
        _say("single", s["n"], s["fn"], s["seed"], s["precision"])
        g = _make(s, precision=s["precision"])
        g.run()
        singles.append(_snapshot(g))
    _say("batch of", len(specs))
    hs = [_make(s, precision=s["precision"]) for s in specs]
    statuses = batch_run(hs)
    assert all(st >= 0 for st in statuses), statuses
    for i, (g, ref) in enumerate(zip(hs, singles)):
        _assert_same(_snapshot(g), ref, i)
    # the same handles again: a second batch starts from scratch
    _say("batch again")
    batch_run(hs)
    for i, (g, ref) in enumerate(zip(hs, singles)):
        _assert_same(_snapshot(g), ref, ("again", i))


def test_fp64_batch_matches_oracle():
    specs = [s for s in _mixed_specs() if s["precision"] == PREC_FP64 and np.prod(s["n"]) <= 70000]
    hs = [_make(s, precision=PREC_FP64) for s in specs]
    _say("fp64 batch of", len(specs))
    batch_run(hs)
    for s, g in zip(specs, hs):
        _say("oracle", s["n"], s["fn"], s["seed"])
        o = Oracle(s["n"], s["eps"], s["fn"], s["params"], seed=s["seed"])
        o.run()
        assert list(g.ranks()) == list(o.ranks())
        for k in range(1, g.d):
            gr, gc = g.pivots(k)
            orows, ocols, *_ = o.pivots(k)
            assert np.array_equal(gr, orows) and np.array_equal(gc, ocols)
        a, b = g.cores_flat(), o.cores_flat()
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))


def test_batch_beyond_one_launch():
    """More problems than one launch names: the rounds are split."""
    specs = [{"n": [16, 16, 16], "eps": 1e-8, "fn": FN_HILBERT, "params": [0.5 + 0.01 * i], "seed": i}
             for i in range(600)]
    _say("batch of", len(specs))
    hs = [_make(s, precision=PREC_FP64) for s in specs]
    batch_run(hs)
    for i in (0, 1, 255, 511, 512, 513, 599):
        g = _make(specs[i], precision=PREC_FP64)
        g.run()
        _assert_same(_snapshot(hs[i]), _snapshot(g), i)


def test_batch_mix_subset_equals_single_solves():
    """The first problems of the mixed 512-problem batch (FP32 sweeps by the
    precision policy at eps = 1e-6), at their full sizes."""
    specs = batch_mix()[:40]
    conv = [{"n": p.n, "eps": p.eps, "fn": p.fn_id, "params": p.params, "seed": p.seed, "grid": p.grid}
            for p in specs]
    _say("batch of", len(conv))
    hs = [_make(s) for s in conv]
    batch_run(hs)
    for i, s in enumerate(conv):
        if i % 4:
            continue
        _say("single", s["n"], s["fn"], s["seed"])
        g = _make(s)
        g.run()
        _assert_same(_snapshot(hs[i]), _snapshot(g), i)
        assert g.stats()["precision_used"] == PREC_FP32


def test_fp32_policy_escalates_to_fp64_alike_in_batch_and_alone():
    """Problem 190 of the mixed batch (5D Hilbert, n = 128, eps = 1e-6) misses
    eps after FP32 sweeps on the sampled-error check and is solved again with
    FP64 sweeps (the precision policy); problem 0 does not.  Alone and in a
    batch the outcome is the same bit for bit."""
    mix = batch_mix()
    picks = [190, 0, 3]
    conv = [{"n": mix[i].n, "eps": mix[i].eps, "fn": mix[i].fn_id, "params": mix[i].params, "seed": mix[i].seed,
             "grid": mix[i].grid} for i in picks]
    singles = []
    for s in conv:
        _say("single", s["n"], s["fn"], s["seed"])
        g = _make(s)
        g.run()
        singles.append((_snapshot(g), g.stats()))
    st190 = singles[0][1]
    assert st190["escalated"] == 1 and st190["precision_used"] == PREC_FP64
    assert 0 <= st190["sampled_err"] <= conv[0]["eps"] and st190["status"] == 0
    for _snap, st in singles[1:]:
        assert st["escalated"] == 0 and st["precision_used"] == PREC_FP32 and 0 <= st["sampled_err"] <= 1e-6
    _say("batch")
    hs = [_make(s) for s in conv]
    batch_run(hs)
    for i, (g, (ref, st)) in enumerate(zip(hs, singles)):
        _assert_same(_snapshot(g), ref, i)
        gs = g.stats()
        assert gs["escalated"] == st["escalated"] and gs["sampled_err"] == st["sampled_err"]


def test_verify_off_and_forced():
    spec = {"n": [16] * 4, "eps": 1e-9, "fn": FN_HILBERT, "params": [1.0], "seed": 5}
    g = _make(spec, precision=PREC_FP64, verify=0)
    g.run()
    assert g.stats()["sampled_err"] == -1.0
    g = _make(spec, precision=PREC_FP64, verify=50000)
    g.run()
    st = g.stats()
    assert 0 <= st["sampled_err"] <= 1e-9 and st["escalated"] == 0
    o = Oracle(spec["n"], spec["eps"], spec["fn"], spec["params"], seed=spec["seed"])
    o.run()
    assert abs(st["sampled_err"] - o.sampled_error(50000)) <= 1e-2 * st["sampled_err"] + 1e-15


def test_batch_statuses_in_one_call_match_stats():
    """tt_batch_statuses returns each problem's tt_stats.status: converged
    problems and problems held below eps by a rank cap, in one batch."""
    from paper_2407_11290_amd import NOT_CONVERGED
    specs = [{"n": [12, 14, 10], "eps": 1e-9, "fn": FN_HILBERT, "params": [1.0], "seed": s} for s in range(4)]
    hs = [_make(s, precision=PREC_FP64) for s in specs]
    hs += [TTCross(s["n"], s["eps"], s["fn"], s["params"], seed=s["seed"], precision=PREC_FP64, r_max=2)
           for s in specs[:2]]
    sts = batch_run(hs)
    assert sts == [g.stats()["status"] for g in hs]
    assert sts[:4] == [0] * 4 and sts[4:] == [NOT_CONVERGED] * 2
