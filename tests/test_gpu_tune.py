"""Tile shapes and the autotuner: a solve ends bit for bit the same under any
tile shape (entries are computed one by one in a fixed order and tile-local
pivots are combined with the lowest-position tie-break), so the tuner may pick
any shape; handles with default tile options then use the tuned one."""
import numpy as np
import pytest

from paper_2407_11290_amd import EINVAL, FN_BIMAXWELL, FN_HILBERT, PREC_FP32, PREC_FP64, TTError
from paper_2407_11290_amd.api import TTCross, batch_autotune, batch_run, tile_table, tile_table_clear

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _bimax(seed):
    rng = np.random.default_rng(seed)
    p = []
    for _ in range(2):
        p += [rng.uniform(0.5, 2.0), *rng.uniform(-2.0, 2.0, 3), rng.uniform(0.5, 2.0)]
    return list(p) + [8.0]


def _snap(g):
    st = g.stats()
    return (st["status"], list(g.ranks()), st["sweeps"], st["pivoted"], st["evaluated"], st["rms"],
            [tuple(map(bytes, g.pivots(k))) for k in range(1, g.d)],
            [g.history(k).tobytes() for k in range(1, g.d)], g.cores_flat().tobytes())


CASES = [
    ("hilbert4d", [24, 40, 17, 33], 1e-9, FN_HILBERT, [1.5], [2, 3, 1, 2], PREC_FP64),
    ("bimax5d", [12, 20, 32, 32, 32], 1e-10, FN_BIMAXWELL, _bimax(4), [1, 2, 2, 2, 2], PREC_FP64),
    ("hilbert5d_fp32", [40] * 5, 1e-6, FN_HILBERT, [0.5], [2] * 5, PREC_FP32),
]
SHAPES = [(8, 8), (8, 64), (16, 32), (64, 16), (128, 64), (256, 8)]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_results_do_not_depend_on_tile_shape(case):
    name, n, eps, fn, params, grid, prec = case
    tile_table_clear()
    _say(name, "default tiles")
    g = TTCross(n, eps, fn, params, seed=11, grid=grid, precision=prec)
    g.run()
    ref = _snap(g)
    ran = 0
    for tr, tc in SHAPES:
        _say(name, "tiles", tr, tc)
        h = TTCross(n, eps, fn, params, seed=11, grid=grid, precision=prec, tile_rows=tr, tile_cols=tc)
        try:
            h.run()
        except TTError as e:
            # a tall tile at rank cap 64 may not fit in one workgroup's LDS
            assert e.code == EINVAL and "LDS" in str(e), str(e)
            continue
        ran += 1
        assert _snap(h) == ref, (tr, tc)
        assert all(t[0] == tr for t in h.tiles())
    assert ran >= 4


def test_autotune_records_a_shape_that_later_handles_use():
    tile_table_clear()
    n, grid = [32, 48, 40, 32], [2, 2, 2, 2]
    g = TTCross(n, 1e-9, FN_HILBERT, [1.0], seed=2, grid=grid, precision=PREC_FP64)
    _say("autotune", n)
    tr, tc, ms = g.autotune(reps=2)
    assert ms > 0
    tab = tile_table()
    assert len(tab) == 1
    e = tab[0]
    assert e["n"] == n and e["grid"] == grid and e["fp32"] == 0 and e["hilbert"] == 1 and e["r_max"] == 64
    assert (e["tile_rows"], e["tile_cols"]) == (tr, tc)
    # the handle's own options are untouched: a default solve equals a fresh one
    g.run()
    h = TTCross(n, 1e-9, FN_HILBERT, [1.0], seed=2, grid=grid, precision=PREC_FP64)
    h.run()
    assert _snap(g) == _snap(h)
    if (tr, tc) != (0, 0):
        assert all(t[0] == tr and t[1] <= tc for t in h.tiles())
    # another class is not affected
    o = TTCross([32, 48, 40], 1e-9, FN_HILBERT, [1.0], seed=2, grid=[2, 2, 2], precision=PREC_FP64)
    o.run()
    tile_table_clear()
    o2 = TTCross([32, 48, 40], 1e-9, FN_HILBERT, [1.0], seed=2, grid=[2, 2, 2], precision=PREC_FP64)
    o2.run()
    assert o.tiles() == o2.tiles()


def test_batch_autotune_then_batch_equals_single_solves():
    tile_table_clear()
    specs = []
    for i in range(6):
        specs.append(dict(n=[32] * 4, eps=1e-6, fn=FN_HILBERT, params=[0.3 * i], seed=i))
        specs.append(dict(n=[16] * 5, eps=1e-6, fn=FN_BIMAXWELL, params=_bimax(i), seed=50 + i))
        specs.append(dict(n=[64] * 3, eps=1e-8, fn=FN_HILBERT, params=[0.1 * i], seed=90 + i))

    def make():
        return [TTCross(s["n"], s["eps"], s["fn"], s["params"], seed=s["seed"], grid=[2] * len(s["n"]))
                for s in specs]

    # reference: one at a time with default tiles
    singles = []
    for g in make():
        g.run()
        singles.append(_snap(g))
    hs = make()
    _say("batch autotune", len(hs))
    assert batch_autotune(hs, reps=1, per_class=3) == 3
    tab = tile_table()
    assert len(tab) == 3
    _say("tuned", [(e["n"], e["tile_rows"], e["tile_cols"]) for e in tab])
    batch_run(hs)
    for i, (g, ref) in enumerate(zip(hs, singles)):
        assert _snap(g) == ref, i
    tuned = {(tuple(e["n"]), e["hilbert"]): (e["tile_rows"], e["tile_cols"]) for e in tab}
    for s, g in zip(specs, hs):
        tr, tc = tuned[(tuple(s["n"]), 1 if s["fn"] == FN_HILBERT else 0)]
        if (tr, tc) != (0, 0) and not g.stats()["escalated"]:
            assert all(t[0] == tr and t[1] <= tc for t in g.tiles())
    tile_table_clear()
