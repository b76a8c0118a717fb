"""Pins of the oracle's restarts after false convergence (not in the paper:
the paper's guards are the random start of Alg. 1, Sec. 2.3, and the sampled
error of Sec. 5).  Each test checks a property fixed independently of the
oracle's own code: exact ranks of a separable sum, brute-force errors, the
worst sample recomputed with numpy, nestedness of the index sets (eq.
nestedpivots) and the pivot residuals recomputed by a dense elimination."""
import itertools

import numpy as np
import pytest

from oracle import Oracle, fn_eval, sample_indices
from oracle.oracle import FN_HILBERT, FN_MAXWELL, FN_MAXWELL_IL, FN_SEPSUM

R_CHECK = 4096


def _two_blocks(n, A=1.0, B=2.0):
    """A on the block of indices all below n_j/2, B on the block all at or
    above it: an exact rank-2 separable sum whose two blocks no cross through
    one of them can see."""
    params = [2.0]
    for c, low in ((A, True), (B, False)):
        for j, m in enumerate(n):
            v = [1.0 if ((i < m // 2) == low) else 0.0 for i in range(m)]
            params += [c * x for x in v] if j == 0 else v
    return np.array(params)


def _framed_two_blocks(n, A=1.0, B=2.0):
    """g(i_1) h(i_d) times the two-block tensor of the middle modes: rank 1
    in the two end unfoldings, rank 2 in the others."""
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


def _assert_nested(o):
    """eq. (nestedpivots), and every unfolding's cross square."""
    d = o.d
    for k in range(1, d):
        rows, cols, _, _, _ = o.pivots(k)
        assert rows.shape[0] == cols.shape[0] == int(o.ranks()[k])
        assert len({tuple(t) for t in rows}) == rows.shape[0]
        assert len({tuple(t) for t in cols}) == cols.shape[0]
    for k in range(1, d - 1):
        Ik = {tuple(t) for t in o.pivots(k)[0]}
        assert all(tuple(t[:-1]) in Ik for t in o.pivots(k + 1)[0])
        Jk1 = {tuple(t) for t in o.pivots(k + 1)[1]}
        assert all(tuple(t[1:]) in Jk1 for t in o.pivots(k)[1])


@pytest.mark.parametrize("n", [[16, 16, 16], [12, 10, 14, 8]])
def test_two_block_tensor_recovered_by_one_restart(n):
    p = _two_blocks(n)
    plain = Oracle(n, 1e-8, FN_SEPSUM, p, seed=0)
    plain.run()
    st, err0 = plain.verify(R_CHECK)
    assert st == 2 and list(plain.ranks()) == [1] * (len(n) + 1) and err0 > 0.1
    o = Oracle(n, 1e-8, FN_SEPSUM, p, seed=0, restarts=3, restart_R=R_CHECK)
    assert o.run() == 0
    info = o.restart_info()
    assert info["used"] == 1 and info["cause"] == 0 and info["err"] <= 1e-8
    # exact TT rank 2 in every unfolding, reproduced to rounding
    assert list(o.ranks()) == [1] + [2] * (len(n) - 1) + [1]
    full, mx = o.full_error()
    assert full <= 1e-14 and mx <= 1e-14 * 2.0
    _assert_nested(o)
    # the seed is the worst sample of the first run, recomputed here: the
    # largest |X - X~| over the check stream (lowest sample on ties)
    idx = sample_indices(n, 1, R_CHECK).reshape(R_CHECK, len(n))
    e = np.abs(plain.fn(idx) - plain.tt_eval(idx))
    worst = int(np.lexsort((np.arange(R_CHECK), -e))[0])
    assert list(info["seeds"][0]) == list(idx[worst])


def test_restarts_off_and_unneeded_change_nothing():
    """A run that meets eps is the same with restarts on; restarts off is the
    plain run."""
    for n, fn, eps in (([9, 8, 10, 7], FN_HILBERT, 1e-9), ([12] * 6, FN_MAXWELL, 1e-6)):
        a = Oracle(n, eps, fn, seed=1)
        a.run()
        b = Oracle(n, eps, fn, seed=1, restarts=4, restart_R=R_CHECK)
        assert b.run() == a.status
        assert b.restart_info()["used"] == 0
        assert np.array_equal(a.ranks(), b.ranks())
        assert np.array_equal(a.cores_flat(), b.cores_flat())


@pytest.mark.parametrize("n,seed", [([16] * 6, 0), ([16] * 6, 2), ([24] * 6, 1)])
def test_interleaved_maxwellian_meets_eps_after_restarts(n, seed):
    """x1,v1,x2,v2,x3,v3: the greedy cross stops at rank 1 with a large
    sampled error; the restarts reach eps, and an independent check stream
    agrees."""
    eps = 1e-6
    plain = Oracle(n, eps, FN_MAXWELL_IL, seed=seed)
    plain.run()
    st, err0 = plain.verify(R_CHECK)
    assert st == 2 and err0 > 0.1 and list(plain.ranks()) == [1] * 7
    o = Oracle(n, eps, FN_MAXWELL_IL, seed=seed, restarts=8, restart_R=R_CHECK)
    assert o.run() == 0
    info = o.restart_info()
    assert info["cause"] == 0 and 1 <= info["used"] <= 8 and info["err"] <= eps
    _assert_nested(o)
    assert o.sampled_error(20000, seed=seed + 7) <= 3 * eps
    # v3 is a separable factor: unfolding 5 has rank 1, its residual is zero
    # after i0, and every restart point was trimmed to i0's v3
    i0 = o.stats()["i0"]
    for pt in info["seeds"]:
        assert pt[5] == i0[5]


def test_maxwellian_mode_orders_are_the_same_tensor():
    """The interleaved function is the natural one with its modes permuted."""
    n_nat = [6, 5, 7, 4, 8, 3]                 # x1, x2, x3, v1, v2, v3
    perm = [0, 3, 1, 4, 2, 5]                  # x1, v1, x2, v2, x3, v3
    n_il = [n_nat[j] for j in perm]
    idx = np.array(list(itertools.product(*[range(m) for m in n_il])), dtype=np.int32)
    nat = idx[:, np.argsort(perm)]
    assert np.array_equal(fn_eval(FN_MAXWELL_IL, n_il, idx), fn_eval(FN_MAXWELL, n_nat, nat))


def test_initial_pivot_residuals_are_the_dense_elimination():
    """After restarts, the recorded residual at each pivot equals the one a
    dense elimination of the superblock X(I_{<=k-1} x [n_k], [n_{k+1}] x
    J_{>k+1}) gives, pivots taken in order (to rounding)."""
    n = [16] * 6
    o = Oracle(n, 1e-6, FN_MAXWELL_IL, seed=0, restarts=8, restart_R=R_CHECK)
    o.run()
    d = o.d
    for k in range(1, d):
        pre = o.pivots(k - 1)[0] if k >= 2 else np.zeros((1, 0), dtype=np.int32)
        suf = o.pivots(k + 1)[1] if k <= d - 2 else np.zeros((1, 0), dtype=np.int32)
        rows = [list(p) + [i] for p in pre for i in range(n[k - 1])]
        cols = [[i] + list(q) for q in suf for i in range(n[k])]
        X = fn_eval(FN_MAXWELL_IL, n, np.array([r + c for r in rows for c in cols], dtype=np.int32)).reshape(
            len(rows), len(cols))
        _, _, rho, gam, piv = o.pivots(k)
        E = X.copy()
        for z in range(len(rho)):
            pz = E[rho[z], gam[z]]
            assert abs(pz - piv[z]) <= 1e-10 * np.max(np.abs(X))
            E = E - np.outer(E[:, gam[z]], E[rho[z], :] / pz)


@pytest.mark.parametrize("n", [[6, 8, 8, 8, 8, 5], [5, 6, 7, 6, 4]])
def test_trimmed_restart_point_on_framed_blocks(n):
    """The worst sample enters the end unfoldings, where the residual is
    exactly zero (rank 1): it is trimmed to i0's end indices, enters only the
    middle unfoldings, and the restart recovers the exact ranks."""
    p = _framed_two_blocks(n)
    o = Oracle(n, 1e-8, FN_SEPSUM, p, seed=0, restarts=3, restart_R=R_CHECK)
    assert o.run() == 0
    info = o.restart_info()
    assert info["used"] == 1 and info["cause"] == 0
    d = len(n)
    assert list(o.ranks()) == [1, 1] + [2] * (d - 3) + [1, 1]
    i0 = o.stats()["i0"]
    assert info["seeds"][0][0] == i0[0] and info["seeds"][0][d - 1] == i0[d - 1]
    full, _ = o.full_error()
    assert full <= 1e-14
    _assert_nested(o)
