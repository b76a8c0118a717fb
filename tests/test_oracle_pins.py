"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
library routines (LAPACK complete-pivoting LU, numpy solves and SVDs), physical
moments of the Maxwellians, brute force on tiny tensors, and the values the
paper prints.  All run on the CPU.
"""
import fractions
import itertools
import os

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle import Oracle, fn_eval, matrix_residual, mix64, pairwise_sumsq, sample_indices, splitmix64, tt_eval
from oracle.oracle import FN_BIMAXWELL, FN_HILBERT, FN_MAXWELL, FN_MAXWELL_2D2V, FN_MAXWELL_3D3V, FN_SEPSUM


def _sepsum_params(n, r, seed):
    rng = np.random.default_rng(seed)
    g = 0.5 + rng.random(r * int(np.sum(n)))
    return np.concatenate([[float(r)], g])


def _full_tensor(fn_id, n, params=None):
    idx = np.array(list(itertools.product(*[range(m) for m in n])), dtype=np.int32)
    return fn_eval(fn_id, n, idx, params).reshape(n)


# --------------------------------------------------------------------------
# Seeded inputs
# --------------------------------------------------------------------------
def test_splitmix64_published_outputs(golden_dir):
    lines = [ln.strip() for ln in open(os.path.join(golden_dir, "splitmix64_seed0.txt"))
             if ln.strip() and not ln.startswith("#")]
    want = [int(x, 16) for x in lines]
    got = [int(x) for x in splitmix64(0, len(want))]
    assert got == want


def test_pairwise_sumsq_against_exact_rational_sum():
    """The sample norm's pairwise sum of squares is within the pairwise
    summation error bound (about log2(n) ulps) of the exact sum, and is exact
    on values whose squares are exactly representable integers."""
    rng = np.random.default_rng(4)
    for n in (1, 2, 3, 1000, 16384, 20000):
        v = rng.standard_normal(n)
        exact = sum(fractions.Fraction(float(x)) ** 2 for x in v)
        got = pairwise_sumsq(v)
        assert abs(fractions.Fraction(got) - exact) <= exact * (np.log2(max(n, 2)) + 2) * 2.0 ** -52
    ints = np.arange(1, 1001, dtype=np.float64)
    assert pairwise_sumsq(ints) == float(sum(int(x) ** 2 for x in ints))
    # padding: the tree over 3 values is (a^2 + b^2) + (c^2 + 0)
    a, b, c = 0.1, 0.7, 1.3
    assert pairwise_sumsq([a, b, c]) == (a * a + b * b) + (c * c + 0.0)


def test_sample_indices_are_in_range_and_stream_ordered():
    n = [5, 7, 3]
    idx = sample_indices(n, 11, 1000)
    assert idx.shape == (1000, 3)
    assert (idx >= 0).all() and (idx < np.array(n)).all()
    draws = splitmix64(11, 3000).reshape(1000, 3)
    assert (idx == (draws % np.array(n, dtype=np.uint64)).astype(np.int32)).all()


# --------------------------------------------------------------------------
# Generating functions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("d,n,shift", [(3, 32, None), (2, 100, None), (6, 9, None), (4, 8, 2.0)])
def test_hilbert_entries_are_correctly_rounded_reciprocals(d, n, shift):
    """eq. (HilbertTensor): 1/(1-d+sum i_j), 1-based; exact rational rounded once."""
    rng = np.random.default_rng(d * 100 + n)
    idx = rng.integers(0, n, size=(500, d)).astype(np.int32)
    params = None if shift is None else [shift]
    got = fn_eval(FN_HILBERT, [n] * d, idx, params)
    s = (1 - d) if shift is None else shift
    for row, g in zip(idx, got):
        den = fractions.Fraction(int(row.sum()) + d) + fractions.Fraction(s)
        assert g == float(1 / den)


def _velocity_moments(fn_id, n, params, spatial_idx, vmax=8.0):
    """Discrete moments over the cell-centred velocity grid on [-vmax, vmax]."""
    nv = n[-3:]
    grids = [-vmax + (np.arange(m) + 0.5) * (2 * vmax / m) for m in nv]
    vv = np.array(list(itertools.product(*[range(m) for m in nv])), dtype=np.int32)
    idx = np.concatenate([np.tile(np.array(spatial_idx, dtype=np.int32), (vv.shape[0], 1)), vv], axis=1)
    f = fn_eval(fn_id, n, idx, params)
    dv3 = np.prod([2 * vmax / m for m in nv])
    V = np.stack([grids[c][vv[:, c]] for c in range(3)], axis=1)
    m0 = f.sum() * dv3
    m1 = (f[:, None] * V).sum(axis=0) * dv3
    return m0, m1, V, f, dv3


def test_maxwellian_moments_at_special_points():
    """Zeroth moment = density, first = density x drift, second = 3 density T.

    At x1 = 1/4, x2 = 0 the density is 1 + a = 1.5; at x3 = 1/4 the drift is
    b = 0.3; at x1 = 0 the density is 1.  These pin the density, drift,
    temperature, normalisation power and exponent of the Maxwellian."""
    n = [8, 8, 8, 48, 48, 48]
    m0, m1, V, f, dv3 = _velocity_moments(FN_MAXWELL, n, None, [2, 0, 2])   # x=(1/4,0,1/4)
    assert abs(m0 - 1.5) < 1e-10
    assert abs(m1[0] / m0 - 0.3) < 1e-10 and abs(m1[1]) < 1e-12 and abs(m1[2]) < 1e-12
    u = np.array([0.3, 0.0, 0.0])
    m2 = (f * ((V - u) ** 2).sum(axis=1)).sum() * dv3
    assert abs(m2 / (3 * m0) - 1.0) < 1e-9                                  # T = 1
    m0b, m1b, *_ = _velocity_moments(FN_MAXWELL, n, None, [0, 3, 0])        # x1 = 0
    assert abs(m0b - 1.0) < 1e-10 and abs(m1b[0]) < 1e-12
    # params override: a=0.2, b=-0.5, T=2, vmax=12 (tail beyond vmax negligible)
    p = [0.2, -0.5, 2.0, 12.0]
    m0c, m1c, V, f, dv3 = _velocity_moments(FN_MAXWELL, n, p, [2, 0, 2], vmax=12.0)
    assert abs(m0c - 1.2) < 1e-9 and abs(m1c[0] / m0c + 0.5) < 1e-9
    m2c = (f * ((V - np.array([-0.5, 0, 0])) ** 2).sum(axis=1)).sum() * dv3
    assert abs(m2c / (3 * m0c) - 2.0) < 1e-8


def test_bimaxwellian_moments_and_spatial_independence():
    p = [0.7, 1.0, -0.5, 0.25, 0.8, 1.6, -1.2, 0.4, 0.0, 1.3, 12.0]
    n = [4, 5, 48, 48, 48]
    m0, m1, *_ = _velocity_moments(FN_BIMAXWELL, n, p, [1, 3], vmax=12.0)
    assert abs(m0 - (0.7 + 1.6)) < 1e-10
    want = 0.7 * np.array([1.0, -0.5, 0.25]) + 1.6 * np.array([-1.2, 0.4, 0.0])
    assert np.allclose(m1, want, atol=1e-10)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, 48, size=(50, 5)).astype(np.int32)
    idx[:, 0] %= 4
    idx[:, 1] %= 5
    a = fn_eval(FN_BIMAXWELL, n, idx, p)
    idx2 = idx.copy()
    idx2[:, 0] = (idx2[:, 0] + 1) % 4
    idx2[:, 1] = (idx2[:, 1] + 2) % 5
    assert np.array_equal(a, fn_eval(FN_BIMAXWELL, n, idx2, p))


def test_sepsum_is_sum_of_separable_products():
    n = [3, 4, 5]
    params = _sepsum_params(n, 2, 0)
    X = _full_tensor(FN_SEPSUM, n, params)
    g = params[1:].reshape(2, -1)
    offs = np.cumsum([0] + n[:-1])
    ref = sum(np.einsum("i,j,k->ijk", *[g[m, offs[j]:offs[j] + n[j]] for j in range(3)]) for m in range(2))
    assert np.allclose(X, ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("fn_id,n", [(FN_MAXWELL_2D2V, [12, 6, 12, 6]), (FN_MAXWELL_3D3V, [6, 4, 6, 4, 6, 4])])
def test_paper_kinetic_tensors_velocity_symmetry(fn_id, n):
    """Sec. 5.2: f is even under v -> -v (both exponentials swap), and positive."""
    X = _full_tensor(fn_id, n)
    assert (X > 0).all()
    flip = X
    for ax in range(1, len(n), 2):
        flip = np.flip(flip, axis=ax)
    assert np.allclose(X, flip, rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# Matrix cross recursion (d = 2 view)
# --------------------------------------------------------------------------
def test_rank1_recursion_equals_direct_cur_residual():
    """eqs. (matrix_CUR) and (aca_approx_E): eliminating pivots one at a time
    gives A - A(:,J) A(I,J)^{-1} A(I,:)."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((30, 40))
    rows, cols = [3, 17, 8, 25, 0], [5, 33, 12, 2, 39]
    R = matrix_residual(A, rows, cols)
    direct = A - A[:, cols] @ np.linalg.solve(A[np.ix_(rows, cols)], A[rows, :])
    assert np.max(np.abs(R - direct)) < 1e-12 * np.max(np.abs(A))
    # interpolation: residual vanishes on pivot rows and columns
    assert np.max(np.abs(R[rows, :])) < 1e-13 and np.max(np.abs(R[:, cols])) < 1e-13


def test_rank1_recursion_sign_convention():
    """A residual must vanish at its own pivot after one step (the sign fix)."""
    A = np.array([[2.0, 1.0], [4.0, 5.0]])
    R = matrix_residual(A, [1], [1])
    assert abs(R[1, 1]) <= 1e-15 and abs(R[1, 0]) <= 1e-15 and abs(R[0, 1]) <= 1e-15
    assert np.isclose(R[0, 0], 2.0 - 1.0 * 4.0 / 5.0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_d2_greedy_equals_complete_pivoting_lu(seed):
    """Sec. 2.3: greedy pivoting is Gaussian elimination with pivoting; on a
    tie-free matrix the d = 2 cross chooses the same pivots, with the same
    Schur-complement pivot values, as LAPACK's complete-pivoting LU (dgetc2)."""
    m = 12
    params = _sepsum_params([m, m], m, seed)          # sum of m random rank-1 terms: full rank
    A = _full_tensor(FN_SEPSUM, [m, m], params)
    o = Oracle([m, m], 0.0, FN_SEPSUM, params, seed=seed, r_max=m)
    o.run()
    st = o.stats()
    # the sample set covers all 144 entries, so the first pivot is the global argmax
    assert np.abs(A[tuple(st["i0"])]) == np.abs(A).max()
    _, _, rho, gam, piv = o.pivots(1)
    lu, ipiv, jpiv, info = lapack.dgetc2(A)
    rp, cp = list(range(m)), list(range(m))
    lrows, lcols = [], []
    for i in range(m):
        rp[i], rp[ipiv[i]] = rp[ipiv[i]], rp[i]
        cp[i], cp[jpiv[i]] = cp[jpiv[i]], cp[i]
        lrows.append(rp[i])
        lcols.append(cp[i])
    z = len(rho)
    assert z == m
    assert list(rho) == lrows[:z] and list(gam) == lcols[:z]
    assert np.allclose(piv, np.diag(lu)[:z], rtol=1e-10, atol=0)


def test_hilbert_matrix_recursion_stays_accurate_past_rank_12():
    """Fig. 2: on the 100 x 100 Hilbert matrix the recursion keeps improving to
    machine precision, where the explicit inverse of A(I,J) degenerates once
    the rank passes about 12."""
    H = 1.0 / (np.arange(1, 101)[:, None] + np.arange(1, 101)[None, :] - 1)
    nH = np.linalg.norm(H)
    errs = {}
    for r in (10, 20):
        o = Oracle([100, 100], 0.0, FN_HILBERT, seed=0, r_max=r)
        o.run()
        assert o.ranks()[1] == r
        G1, G2 = o.cores()
        rows, cols, *_ = o.pivots(1)
        I, J = rows[:, 0], cols[:, 0]
        resid = matrix_residual(H, I, J)                      # eq. (aca_approx_E)
        direct = H[:, J] @ np.linalg.inv(H[np.ix_(I, J)]) @ H[I, :]
        errs[r] = (np.linalg.norm(resid) / nH, np.linalg.norm(H - G1[0] @ G2[:, :, 0]) / nH,
                   np.linalg.norm(H - direct) / nH)
    # at rank 10 all three agree; at rank 20 only the recursions stay accurate
    assert abs(errs[10][0] - errs[10][2]) < 1e-3 * errs[10][0]
    assert errs[20][0] < 1e-15 and errs[20][1] < 1e-15
    assert errs[20][2] > 1e6 * errs[20][0]


# --------------------------------------------------------------------------
# Tensor cross: definitions and invariants
# --------------------------------------------------------------------------
def _skeleton_check(o):
    """eq. (ttcross_build_elem) interpolates: TT = X on every I_{<=k-1} x [n_k] x J_{>k}."""
    d, n = o.d, o.n
    worst = 0.0
    for k in range(1, d + 1):
        Ik = o.pivots(k - 1)[0] if k >= 2 else np.zeros((1, 0), np.int32)
        Jk = o.pivots(k)[1] if k <= d - 1 else np.zeros((1, 0), np.int32)
        idx = np.array([list(p) + [i] + list(q) for p in Ik for i in range(n[k - 1]) for q in Jk],
                       dtype=np.int32)
        x = o.fn(idx)
        y = o.tt_eval(idx)
        worst = max(worst, np.max(np.abs(x - y)) / np.max(np.abs(x)))
    return worst


def test_sepsum_exact_low_rank_recovery():
    """eq. (matrix_CUR) is exact when rank A(I,J) = rank A: a sum of r separable
    terms gives TT ranks <= r and a reconstruction exact to rounding."""
    n = [7, 9, 8, 6]
    params = _sepsum_params(n, 3, 5)
    o = Oracle(n, 1e-12, FN_SEPSUM, params, seed=3)
    o.run()
    r = o.ranks()
    assert (r[1:-1] <= 3).all() and r[1:-1].max() == 3
    err, mx = o.full_error()
    assert err < 1e-13
    assert _skeleton_check(o) < 1e-13


def test_bimaxwellian_recovered_at_rank_two():
    n = [3, 16, 16, 16]
    p = [0.9, 0.5, -1.0, 0.3, 0.7, 1.4, -0.2, 1.1, -1.5, 1.2, 8.0]
    o = Oracle(n, 1e-10, FN_BIMAXWELL, p, seed=1)
    o.run()
    r = o.ranks()
    assert (r[1:-1] <= 2).all()
    err, _ = o.full_error()
    assert err < 1e-12


def test_ranks_bounded_by_unfolding_ranks():
    """eq. (TT_trivial): r_k <= rank(X_k) (numpy SVD of each unfolding)."""
    n = [4, 5, 6, 5]
    params = _sepsum_params(n, 2, 9)
    X = _full_tensor(FN_SEPSUM, n, params)
    o = Oracle(n, 1e-12, FN_SEPSUM, params, seed=0, r_max=30)
    o.run()
    r = o.ranks()
    for k in range(1, 4):
        Xk = X.reshape(int(np.prod(n[:k])), -1)
        assert r[k] <= np.linalg.matrix_rank(Xk)


def test_hilbert_config1_full_tensor_error_below_eps():
    """eq. (FrobeniusNorm) by brute force over all 32768 entries of the 3D
    Hilbert tensor, n = 32, eps = 1e-10, for ten seeds."""
    for seed in range(10):
        o = Oracle([32, 32, 32], 1e-10, FN_HILBERT, seed=seed)
        o.run()
        err, _ = o.full_error()
        assert err <= 1e-10, (seed, err)
        assert o.stats()["status"] == 0


def test_interpolation_on_skeleton_hilbert():
    o = Oracle([16, 16, 16, 16], 1e-9, FN_HILBERT, seed=4)
    o.run()
    assert _skeleton_check(o) < 1e-11


def test_nested_index_sets():
    """eq. (nestedpivots): I_{<=k+1} in I_{<=k} x [n], J_{>k} in [n] x J_{>k+1}."""
    o = Oracle([10, 11, 12, 13, 9], 1e-9, FN_HILBERT, seed=2)
    o.run()
    d = o.d
    for k in range(1, d - 1):
        Ik = {tuple(t) for t in o.pivots(k)[0]}
        Ik1 = o.pivots(k + 1)[0]
        assert all(tuple(t[:-1]) in Ik for t in Ik1)
    for k in range(1, d - 1):
        Jk = o.pivots(k)[1]
        Jk1 = {tuple(t) for t in o.pivots(k + 1)[1]}
        assert all(tuple(t[1:]) in Jk1 for t in Jk)


def test_cores_match_direct_solve_and_identity_rows():
    """eq. (ttcross_build): G_k = X(I_{<=k-1},:,J_{>k}) X(I_{<=k},J_{>k})^{-1}
    (numpy solve), and Alg. 4's T_k equals the identity on the pivot rows."""
    n = [9, 10, 11, 8]
    params = _sepsum_params(n, 4, 2)
    o = Oracle(n, 1e-13, FN_SEPSUM, params, seed=7)
    o.run()
    d = o.d
    cores = o.cores()
    for k in range(1, d):
        rows, cols, rho, gam, piv = o.pivots(k)
        prev = o.pivots(k - 1)[0] if k >= 2 else np.zeros((1, 0), np.int32)
        S = np.array([[o.fn(np.array(list(p) + [i] + list(q), np.int32))[0] for q in cols]
                      for p in prev for i in range(n[k - 1])])
        P = np.array([[o.fn(np.array(list(a) + list(b), np.int32))[0] for b in cols] for a in rows])
        G = np.linalg.solve(P.T, S.T).T
        Gk = cores[k - 1].reshape(-1, cores[k - 1].shape[2])
        assert np.max(np.abs(G - Gk)) < 1e-9 * max(1.0, np.max(np.abs(G)))
        assert np.max(np.abs(Gk[rho, :] - np.eye(len(rho)))) < 1e-12


def test_superblock_residual_is_the_cur_residual():
    """The residual the greedy search scans is X(R,C) - X(R,J) X(I,J)^{-1} X(I,C)."""
    n = [6, 7, 8, 5]
    params = _sepsum_params(n, 5, 4)
    o = Oracle(n, 0.0, FN_SEPSUM, params, seed=1, r_max=4)
    o.run()
    d = o.d
    for k in range(1, d):
        E = o.superblock_residual(k)
        rows, cols, *_ = o.pivots(k)
        prev = o.pivots(k - 1)[0] if k >= 2 else np.zeros((1, 0), np.int32)
        nxt = o.pivots(k + 1)[1] if k + 1 <= d - 1 else np.zeros((1, 0), np.int32)
        R = [list(p) + [i] for p in prev for i in range(n[k - 1])]
        Cc = [[j] + list(q) for q in nxt for j in range(n[k])]
        X = lambda A, B: np.array([[o.fn(np.array(a + list(b), np.int32))[0] for b in B] for a in A])
        XRC = X(R, Cc)
        XRJ = X(R, [list(c) for c in cols])
        XIJ = X([list(r) for r in rows], [list(c) for c in cols])
        XIC = X([list(r) for r in rows], Cc)
        cur = XRC - XRJ @ np.linalg.solve(XIJ, XIC)
        assert np.max(np.abs(E - cur)) < 1e-11 * np.max(np.abs(XRC))


def test_stop_rule_holds_on_final_superblocks():
    """At a converged stop, no unmasked superblock residual exceeds tau."""
    o = Oracle([12, 12, 12, 12], 1e-7, FN_HILBERT, seed=5)
    o.run()
    st = o.stats()
    assert st["status"] == 0
    for k in range(1, 4):
        E = o.superblock_residual(k)
        _, _, rho, gam, _ = o.pivots(k)
        mask = np.ones_like(E, dtype=bool)
        mask[rho, :] = False
        mask[:, gam] = False
        assert np.abs(E[mask]).max() <= st["tau"]


def test_rank_cap_reports_not_converged():
    o = Oracle([16, 16, 16], 1e-14, FN_HILBERT, seed=0, r_max=4)
    assert o.run() == 1
    assert list(o.ranks()) == [1, 4, 4, 1]


@pytest.mark.slow
def test_paper_table6_hilbert3d_n250_loose(golden_dir):
    """Table 6: rank (1,25,25,1) on the 3D Hilbert tensor, n = 250, gives a
    sampled error of about 1e-6 with the paper's sampled/rook pivoting.  A full
    greedy search picks each pivot at the global residual maximum, so it must do
    at least as well (it reaches rounding level); the pin is one-sided."""
    vals = {}
    for ln in open(os.path.join(golden_dir, "table6_hilbert3d_n250.txt")):
        if ln.strip() and not ln.startswith("#"):
            k, *v = ln.split()
            vals[k] = [float(x) for x in v]
    n = int(vals["n"][0])
    o = Oracle([n, n, n], 0.0, FN_HILBERT, seed=0, r_max=int(vals["ranks"][1]))
    o.run()
    assert list(o.ranks()) == [int(x) for x in vals["ranks"]]
    err = o.sampled_error(1_000_000)
    ref = vals["error_subtensor"][0]
    assert err < ref, err


def test_tt_eval_matches_explicit_matrix_product():
    rng = np.random.default_rng(0)
    n = [3, 4, 2]
    ranks = [1, 2, 3, 1]
    cores = [rng.standard_normal((ranks[k], n[k], ranks[k + 1])) for k in range(3)]
    flat = np.concatenate([c.ravel() for c in cores])
    idx = np.array(list(itertools.product(*[range(m) for m in n])), dtype=np.int32)
    got = tt_eval(n, ranks, flat, idx)
    ref = np.array([(cores[0][:, a, :] @ cores[1][:, b, :] @ cores[2][:, c, :])[0, 0] for a, b, c in idx])
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# Rook mode: Alg. 1 inside every subtensor block, best of the local pivots
# (Alg. 3)
# --------------------------------------------------------------------------
def _piece(i, n, C):
    """Subtensor block of index i when n indices are split evenly into C
    pieces (Sec. 3): the last b with floor(b n / C) <= i."""
    return max(b for b in range(C) if (b * n) // C <= i)


def _pivot_positions(o):
    return [tuple(map(bytes, o.pivots(k)[:2])) for k in range(1, o.d)]


def test_rook_stream_seeds_use_splitmix64_output_function(golden_dir):
    """The per-block sample streams start at seed XOR mix(tag), mix being the
    output function of SplitMix64: applied to 1, 2, 3 times the golden gamma it
    gives the generator's first outputs from state 0."""
    lines = [ln.strip() for ln in open(os.path.join(golden_dir, "splitmix64_seed0.txt"))
             if ln.strip() and not ln.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    for t in range(3):
        assert mix64((gamma * (t + 1)) & 0xFFFFFFFFFFFFFFFF) == int(lines[t], 16)


@pytest.mark.parametrize("n,fn_id,params,seed", [
    ([12, 10, 9], FN_HILBERT, None, 3),
    ([6, 7, 5, 4], FN_HILBERT, [0.5], 1),
    ([7, 6, 8], FN_SEPSUM, "sep", 2),
])
def test_rook_with_single_entry_blocks_is_the_greedy_search(n, fn_id, params, seed):
    """With mode j split into n_j pieces every subtensor block of a superblock
    is one entry, so Alg. 1 returns that entry and the best of the local
    pivots is the full-search (greedy) pivot: pivots, ranks and cores agree bit
    for bit."""
    if params == "sep":
        params = _sepsum_params(n, 4, 9)
    g = Oracle(n, 1e-10, fn_id, params, seed=seed)
    g.run()
    r = Oracle(n, 1e-10, fn_id, params, seed=seed, pivot="rook", grid=n)
    r.run()
    assert list(r.ranks()) == list(g.ranks())
    assert _pivot_positions(r) == _pivot_positions(g)
    assert np.array_equal(r.cores_flat(), g.cores_flat())


@pytest.mark.parametrize("grid,seed", [([1, 1], 0), ([2, 3], 1), ([4, 2], 2)])
def test_rook_pivots_are_rook_pivots_within_their_block(grid, seed):
    """d = 2: every pivot, in order, has the largest |residual| of its row and
    of its column inside its subtensor block (the stopping condition of
    Alg. 1), with the residual from the direct CUR formula
    A - A(:,J) A(I,J)^{-1} A(I,:) over the earlier pivots (numpy solve, not the
    oracle's recursion).  The rook pivots are not all the greedy ones."""
    n = [40, 52]
    params = _sepsum_params(n, 10, 2)
    A = _full_tensor(FN_SEPSUM, n, params)
    o = Oracle(n, 1e-14, FN_SEPSUM, params, seed=seed, pivot="rook", grid=grid)
    o.run()
    _, _, rho, gam, _ = o.pivots(1)
    assert len(rho) == 10
    for z in range(len(rho)):
        I, J = list(rho[:z]), list(gam[:z])
        R = A.copy() if z == 0 else A - A[:, J] @ np.linalg.solve(A[np.ix_(I, J)], A[I, :])
        i, j = int(rho[z]), int(gam[z])
        rows = [r for r in range(n[0]) if _piece(r, n[0], grid[0]) == _piece(i, n[0], grid[0]) and r not in I]
        cols = [c for c in range(n[1]) if _piece(c, n[1], grid[1]) == _piece(j, n[1], grid[1]) and c not in J]
        tol = 1e-10 * np.abs(R).max()
        assert abs(R[i, j]) >= np.abs(R[rows, j]).max() - tol, z
        assert abs(R[i, j]) >= np.abs(R[i, cols]).max() - tol, z
    g = Oracle(n, 1e-14, FN_SEPSUM, params, seed=seed)
    g.run()
    assert _pivot_positions(g) != _pivot_positions(o)


def test_rook_exact_low_rank_recovery_and_interpolation():
    """Exactness of eq. (matrix_CUR) does not depend on which pivots are taken:
    a sum of 3 separable terms is recovered at ranks <= 3 in rook mode too,
    and the TT interpolates the tensor on its skeleton."""
    n = [7, 9, 8, 6]
    params = _sepsum_params(n, 3, 5)
    o = Oracle(n, 1e-12, FN_SEPSUM, params, seed=3, pivot="rook", grid=[2, 3, 1, 2])
    o.run()
    r = o.ranks()
    assert (r[1:-1] <= 3).all() and r[1:-1].max() == 3
    err, _ = o.full_error()
    assert err < 1e-13
    assert _skeleton_check(o) < 1e-13


def test_rook_hilbert3d_full_tensor_error_below_eps():
    """The 3D Hilbert tensor, n = 32, eps = 1e-10, with rook search on a 2x2x2
    block grid: the full-tensor relative error meets eps, and the search looks
    at fewer residuals than the full search."""
    n = [32] * 3
    for seed in (0, 1):
        o = Oracle(n, 1e-10, FN_HILBERT, seed=seed, pivot="rook", grid=[2, 2, 2])
        o.run()
        err, _ = o.full_error()
        assert err <= 1e-10
        g = Oracle(n, 1e-10, FN_HILBERT, seed=seed)
        g.run()
        assert o.stats()["pivoted"] < g.stats()["pivoted"]


def test_prescribed_ranks_cap_each_unfolding():
    """Per-unfolding rank caps (the paper's runs at fixed core ranks, Sec. 5):
    with eps = 0 every unfolding stops at its own cap, the run reports the cap
    as what stopped it, and equal caps reproduce a global rank cap bit for
    bit."""
    n = [12, 10, 9, 8]
    o = Oracle(n, 0.0, FN_HILBERT, seed=2, rank_caps=[5, 3, 7])
    assert o.run() == 1                                   # not converged: stopped by the caps
    assert list(o.ranks()) == [1, 5, 3, 7, 1]
    a = Oracle(n, 0.0, FN_HILBERT, seed=2, rank_caps=[4, 4, 4])
    b = Oracle(n, 0.0, FN_HILBERT, seed=2, r_max=4)
    a.run()
    b.run()
    assert _pivot_positions(a) == _pivot_positions(b)
    assert np.array_equal(a.cores_flat(), b.cores_flat())
    # caps change nothing before an unfolding reaches one (the smallest is
    # 3), so the first two pivots of every unfolding are those of a run with
    # a larger global cap
    c = Oracle(n, 0.0, FN_HILBERT, seed=2, r_max=8)
    c.run()
    for k in range(1, 4):
        assert np.array_equal(o.pivots(k)[2][:2], c.pivots(k)[2][:2])
