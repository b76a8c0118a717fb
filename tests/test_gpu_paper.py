"""The paper's kinetic tensors (Sec. 5.2/5.3, eq. 2d2vFunction and its 3d3v
extension, modes x, v_x, y, v_y[, z, v_z]) at reduced sizes with prescribed
core ranks, GPU against the FP64 oracle.

These tensors are even under v -> -v, so their superblocks hold pairs of
entries that are equal in exact arithmetic and differ only by rounding; the
greedy search then meets near-ties at the 1e-16 level.  The device
exponential may differ from the host's by an ulp, so such a tie can be
decided either way, and the pivot sequences may part there.  What is unique
is compared: the ranks, and every sweep's largest |residual| up to the first
pivot where the two sides differ; that first difference must sit on a near-tie
logged by the oracle (relative gap below 1e-10); and the final sampled
errors must agree to within a factor of two.  A sequence without a
divergence is compared bit for bit in its pivots."""
import numpy as np
import pytest

from oracle import Oracle, fn_eval as orc_fn_eval, sample_indices
from paper_2407_11290_amd import FN_MAXWELL_2D2V, FN_MAXWELL_3D3V, PREC_FP64
from paper_2407_11290_amd.api import TTCross

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _first_divergence(g, o, d):
    """(pivot index z, unfolding k) of the first pivot, in sweep order, where
    the two sides' tuples differ, or None."""
    first = None
    for k in range(1, d):
        gr, gc = g.pivots(k)
        orows, ocols, *_ = o.pivots(k)
        for z in range(min(len(gr), len(orows))):
            if not (np.array_equal(gr[z], orows[z]) and np.array_equal(gc[z], ocols[z])):
                if first is None or z < first[0]:
                    first = (z, k)
                break
    return first


@pytest.mark.parametrize("fn,n,caps", [
    (FN_MAXWELL_2D2V, [24, 12, 24, 12], [10, 5, 12]),
    (FN_MAXWELL_2D2V, [40, 20, 40, 20], [10, 5, 20]),
    (FN_MAXWELL_3D3V, [16, 8, 16, 8, 16, 8], [6, 3, 8, 3, 6]),
])
@pytest.mark.parametrize("seed", [0, 1])
def test_kinetic_tensors_at_prescribed_ranks_against_the_oracle(fn, n, caps, seed):
    d = len(n)
    _say("kinetic", fn, n, caps, seed)
    g = TTCross(n, 0.0, fn, seed=seed, grid=[2] * d, precision=PREC_FP64)
    g.set_rank_caps(caps)
    gs = g.run()
    o = Oracle(n, 0.0, fn, seed=seed, rank_caps=caps)
    os_ = o.run()
    assert gs == os_ == 1                                   # stopped by the prescribed ranks
    assert list(g.ranks()) == list(o.ranks()) == [1] + caps + [1]
    div = _first_divergence(g, o, d)
    last = div[0] - 1 if div else None                     # sweeps identical up to here
    # late residuals are small differences of O(max |X|) entries, so they are
    # compared on the tensor's scale (the first sweep's largest |residual|)
    scale = max(o.history(k)[0] for k in range(1, d))
    for k in range(1, d):
        gh, oh = g.history(k), o.history(k)
        m = min(len(gh), len(oh)) if last is None else min(last + 1, len(gh), len(oh))
        assert np.allclose(gh[:m], oh[:m], rtol=0, atol=1e-12 * scale), k
    if div is None:
        _say("pivots identical")
    elif div[0] == 0:
        # the first pivot is the largest |sample|: two samples whose values
        # differ by rounding (v and -v) may be taken either way
        gi0 = np.concatenate([g.pivots(1)[0][0], g.pivots(1)[1][0]]).astype(np.int32)
        oi0 = o.stats()["i0"].astype(np.int32)
        fg, fo = orc_fn_eval(fn, n, np.stack([gi0, oi0]))
        _say("first pivots differ", gi0, oi0, fg, fo)
        assert abs(abs(fg) - abs(fo)) <= 1e-14 * abs(fo)
    else:
        z, k = div
        gap = o.gap_history(k)[z - 1]
        best = o.history(k)[z - 1]
        _say("first divergence: pivot", z, "of unfolding", k, "oracle gap", gap, "best |residual|", best)
        # a near-tie, or a choice among residuals at the rounding level
        assert gap < 1e-10 or best < 1e-12 * scale
    idx = sample_indices(n, 5, 50000)
    x = orc_fn_eval(fn, n, idx)
    eg = np.sqrt(np.sum((x - g.tt_eval(idx)) ** 2) / np.sum(x ** 2))
    eo = np.sqrt(np.sum((x - o.tt_eval(idx)) ** 2) / np.sum(x ** 2))
    _say("sampled errors gpu", eg, "oracle", eo)
    assert eg <= 2 * eo + 1e-14 and eo <= 2 * eg + 1e-14
