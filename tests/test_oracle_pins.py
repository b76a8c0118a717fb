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


# --------------------------------------------------------------------------
# Error measures: brute-force Frobenius error (eq. FrobeniusNorm) and the
# sampled error of Sec. 5, against numpy on the same cores
# --------------------------------------------------------------------------
def _tt_full_numpy(cores):
    """The full tensor of a TT by explicit contraction of its cores (einsum)."""
    full = cores[0]
    for G in cores[1:]:
        full = np.tensordot(full, G, axes=([full.ndim - 1], [0]))
    return full[0, ..., 0]


def _hilbert_numpy(n, shift=None):
    """eq. (HilbertTensor) in closed form on the 0-based grid: 1/(sum (i_j+1) + shift)."""
    d = len(n)
    s = (1 - d) if shift is None else shift
    grids = np.meshgrid(*[np.arange(m) + 1.0 for m in n], indexing="ij")
    return 1.0 / (sum(grids) + s)


@pytest.mark.parametrize("case", ["hilbert", "sepsum"])
def test_full_and_sampled_error_against_numpy(case):
    """orc_full_error and orc_sampled_error against numpy: the tensor in closed
    form (Hilbert) or as an einsum of separable factors, the TT by contracting
    the oracle's cores, the sampled indices from the published SplitMix64
    stream.  The cases stop at a rank cap, so the errors are far from zero."""
    if case == "hilbert":
        n, params, r_max, fn = [9, 10, 11], None, 3, FN_HILBERT
        X = _hilbert_numpy(n)
    else:
        n, r_max, fn = [6, 7, 5, 8], 2, FN_SEPSUM
        params = _sepsum_params(n, 4, 11)
        g = params[1:].reshape(4, -1)
        offs = np.cumsum([0] + n[:-1])
        X = sum(np.einsum("i,j,k,l->ijkl", *[g[m, offs[j]:offs[j] + n[j]] for j in range(4)]) for m in range(4))
    o = Oracle(n, 1e-14, fn, params, seed=3, r_max=r_max)
    assert o.run() == 1                                   # stopped by the rank cap
    Y = _tt_full_numpy(o.cores())
    want = np.linalg.norm(X - Y) / np.linalg.norm(X)
    assert want > 1e-5                                    # a real error, not rounding
    err, mx = o.full_error()
    assert abs(err - want) <= 1e-10 * want
    assert abs(mx - np.max(np.abs(X - Y))) <= 1e-10 * mx
    R, seed = 20000, 77
    idx = sample_indices(n, seed, R)
    x, y = X[tuple(idx.T)], Y[tuple(idx.T)]
    want_s = np.sqrt(np.sum((x - y) ** 2) / np.sum(x ** 2))
    got_s = o.sampled_error(R, seed)
    assert abs(got_s - want_s) <= 1e-10 * want_s
    # the default stream of the sampled error is seed + 1
    idx1 = sample_indices(n, 4, R)
    x1, y1 = X[tuple(idx1.T)], Y[tuple(idx1.T)]
    assert abs(o.sampled_error(R) - np.sqrt(np.sum((x1 - y1) ** 2) / np.sum(x1 ** 2))) <= 1e-10 * want_s


# --------------------------------------------------------------------------
# Tie-break: among equal |residual| the lowest (row position, column
# position) wins
# --------------------------------------------------------------------------
def _matrix_as_sepsum(A):
    """A d = 2 separable sum of m terms that is exactly the m x n matrix A:
    term m is e_m(i) A(m, j) (products with 0 and 1 and sums of zeros are
    exact)."""
    m, n = A.shape
    params = [float(m)]
    for t in range(m):
        params += [1.0 if i == t else 0.0 for i in range(m)] + list(A[t])
    return np.array(params)


def test_tie_break_lowest_row_then_column_on_a_hand_built_matrix():
    """A 6 x 6 matrix whose first pivot (10 at (0,0)) is unique and whose
    other nonzeros sit in rows and columns that no elimination touches, so
    the residual keeps exact ties at |5|: the pivots must come in the order
    (1,4) before (1,5) (same row, lower column), then (2,3), (3,1), (4,2)
    (lower rows first), whatever the signs."""
    A = np.zeros((6, 6))
    A[0, 0] = 10.0
    A[1, 4], A[1, 5] = -5.0, 5.0
    A[2, 3] = 5.0
    A[3, 1] = -5.0
    A[4, 2] = 5.0
    A[5, 5] = 1.0
    o = Oracle([6, 6], 1e-12, FN_SEPSUM, _matrix_as_sepsum(A), seed=0, r_max=6)
    o.run()
    _, _, rho, gam, piv = o.pivots(1)
    assert list(zip(rho, gam))[:5] == [(0, 0), (1, 4), (2, 3), (3, 1), (4, 2)]
    assert list(piv[:5]) == [10.0, -5.0, 5.0, -5.0, 5.0]


def _greedy_tt_cross_numpy(n, fn, eps, seed, r_max=64, tie="low"):
    """A second, independent greedy TT cross in numpy for tiny tensors: the
    same readings as the oracle (samples, first pivot, Jacobi sweeps,
    stop rule, masks), residuals by numpy's elementwise rank-1 updates (two
    roundings, not one fma).  tie = "low" takes the lowest (row, column)
    among equal |residual|, "high" the highest.  Returns the pivot tuples
    and the number of searches in which the largest |residual| was tied."""
    d = len(n)
    idx = sample_indices(n, seed, 16384)
    v = fn(idx)
    rms = np.sqrt(pairwise_sumsq(v) / v.size)
    tau = eps * rms
    i0 = tuple(int(x) for x in idx[int(np.argmax(np.abs(v)))])
    I = {k: [i0[:k]] for k in range(1, d)}
    J = {k: [i0[k:]] for k in range(1, d)}
    I[0], J[d] = [()], [()]
    rho = {k: [i0[k - 1]] for k in range(1, d)}
    gam = {k: [i0[k]] for k in range(1, d)}
    ties = 0
    while True:
        props = {}
        snapI = {k: list(I[k]) for k in I}
        snapJ = {k: list(J[k]) for k in J}
        for k in range(1, d):
            rows = [p + (i,) for p in snapI[k - 1] for i in range(n[k - 1])]
            cols = [(j,) + q for q in snapJ[k + 1] for j in range(n[k])]
            E = fn(np.array([r + c for r in rows for c in cols], dtype=np.int32)).reshape(len(rows), len(cols))
            for pr, pc in zip(rho[k], gam[k]):
                E = E - np.outer(E[:, pc], E[pr, :] / E[pr, pc])
            A = np.abs(E)
            A[rho[k], :] = -1.0
            A[:, gam[k]] = -1.0
            best = A.max()
            where = np.argwhere(A == best)                 # row-major order
            ties += len(where) > 1
            r, c = where[0] if tie == "low" else where[-1]
            if best > tau and len(rho[k]) < r_max:
                props[k] = (int(r), int(c))
        if not props:
            break
        for k, (r, c) in props.items():
            I[k].append(snapI[k - 1][r // n[k - 1]] + (r % n[k - 1],))
            J[k].append((c % n[k],) + snapJ[k + 1][c // n[k]])
            rho[k].append(r)
            gam[k].append(c)
    return {k: (I[k], J[k]) for k in range(1, d)}, ties


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tie_break_on_hilbert_duplicate_rows(seed):
    """The 3D Hilbert tensor's superblocks have bitwise-equal rows (entries
    depend on index sums only), so the largest |residual| is tied exactly in
    many searches.  An independent numpy greedy cross with the lowest-position
    rule reproduces the oracle's pivot tuples; with the highest-position rule
    it does not, so the rule decides the result."""
    n, eps = [12, 12, 12], 1e-10
    fn = lambda idx: fn_eval(FN_HILBERT, n, idx)
    o = Oracle(n, eps, FN_HILBERT, seed=seed)
    o.run()
    low, ties = _greedy_tt_cross_numpy(n, fn, eps, seed, tie="low")
    assert ties > 0
    for k in (1, 2):
        rows, cols, *_ = o.pivots(k)
        assert [tuple(t) for t in rows] == low[k][0], k
        assert [tuple(t) for t in cols] == low[k][1], k
    high, _ = _greedy_tt_cross_numpy(n, fn, eps, seed, tie="high")
    assert any(high[k] != low[k] for k in (1, 2))


# --------------------------------------------------------------------------
# Kinetic tensors of Sec. 5.2 (eq. 2d2vFunction): velocity moments at the
# special points x = +-1/4, where sin(2 pi x) = +-1
# --------------------------------------------------------------------------
def _trunc_gauss(mu, T, a=-3.0, b=3.0):
    """Mass, mean and second moment of exp(-(v-mu)^2/(2T)) on [a, b]
    (standard truncated-normal formulas, scipy's normal cdf and pdf)."""
    from scipy.stats import norm
    s = np.sqrt(T)
    al, be = (a - mu) / s, (b - mu) / s
    Z = norm.cdf(be) - norm.cdf(al)
    mass = np.sqrt(2 * np.pi * T) * Z
    m1 = mu + s * (norm.pdf(al) - norm.pdf(be)) / Z
    var = T * (1 + (al * norm.pdf(al) - be * norm.pdf(be)) / Z - ((norm.pdf(al) - norm.pdf(be)) / Z) ** 2)
    return mass, m1, var + m1 ** 2


def _kinetic_moments(fn_id, n, xs_idx, nv):
    """Midpoint-rule velocity moments of the oracle's tensor at fixed spatial
    indices: mass, <v_1>, <v_1^2>, <v_1 v_2> (normalised by the mass)."""
    ndim = len(xs_idx)
    vgrid = -3.0 + (np.arange(nv) + 0.5) * (6.0 / nv)
    vv = np.array(list(itertools.product(range(nv), repeat=ndim)), dtype=np.int32)
    idx = np.zeros((vv.shape[0], 2 * ndim), dtype=np.int32)
    for w in range(ndim):
        idx[:, 2 * w] = xs_idx[w]
        idx[:, 2 * w + 1] = vv[:, w]
    f = fn_eval(fn_id, n, idx)
    h = (6.0 / nv) ** ndim
    V = vgrid[vv]
    mass = f.sum() * h
    return (mass, (f * V[:, 0]).sum() * h / mass, (f * V[:, 0] ** 2).sum() * h / mass,
            (f * V[:, 0] * V[:, 1]).sum() * h / mass)


@pytest.mark.parametrize("fn_id,nx,nv,tol", [(FN_MAXWELL_2D2V, 6, 1000, 2e-6), (FN_MAXWELL_3D3V, 6, 160, 2e-4)])
def test_paper_kinetic_tensors_velocity_moments(fn_id, nx, nv, tol):
    """eq. (2d2vFunction) at x_w = +-1/4 (cell centres of [-1/2, 1/2] when
    n = 6): rho = 1 +- 0.875, T = 0.5 +- 0.4.  In velocity f is an equal
    mixture of two Gaussians of variance T(x_w) per axis, centred at
    (0.75, .., 0.75) and (-0.75, .., -0.75) and cut to [-3, 3]; the mass is
    prefactor x 2 x prod_w (truncated Gaussian mass), the prefactor being
    sum_w rho(x_w) / (2 sqrt(2 pi T(x_w))).  Closed forms from the
    truncated-normal moments; the tensor's sums are midpoint rules, hence
    the tolerances."""
    ndim = 2 if fn_id == FN_MAXWELL_2D2V else 3
    n = [nx, nv] * ndim
    x_of = {1: -0.25, 4: 0.25}                     # cell centres -1/2 + (i + 1/2)/6
    rho_T = {-0.25: (1 - 0.875, 0.5 - 0.4), 0.25: (1 + 0.875, 0.5 + 0.4)}
    for xs_idx in ([4] * ndim, [4, 1] + [4] * (ndim - 2), [1] * ndim):
        rT = [rho_T[x_of[i]] for i in xs_idx]
        mass, m1, m2, m12 = _kinetic_moments(fn_id, n, xs_idx, nv)
        pre = sum(r / (2 * np.sqrt(2 * np.pi * T)) for r, T in rT)
        gp = [_trunc_gauss(0.75, T) for _, T in rT]
        gm = [_trunc_gauss(-0.75, T) for _, T in rT]
        want_mass = pre * (np.prod([g[0] for g in gp]) + np.prod([g[0] for g in gm]))
        # by symmetry of [-3, 3] both components have the same mass
        assert abs(mass - want_mass) <= tol * want_mass, (xs_idx, mass, want_mass)
        assert abs(m1) <= tol                                       # the two drifts cancel
        want_m2 = 0.5 * (gp[0][2] + gm[0][2])
        assert abs(m2 - want_m2) <= tol * want_m2, (xs_idx, m2, want_m2)
        want_m12 = 0.5 * (gp[0][1] * gp[1][1] + gm[0][1] * gm[1][1])
        assert abs(m12 - want_m12) <= tol * abs(want_m12), (xs_idx, m12, want_m12)
        assert want_m12 > 0                                         # drifts share their sign


# --------------------------------------------------------------------------
# Rook mode: Alg. 1's loop runs until neither step moves
# --------------------------------------------------------------------------
def _bidiagonal(n):
    """Values rise along the staircase (0,0) < (0,1) < (1,1) < (1,2) < ..:
    each row's largest entry is its superdiagonal one and each column's its
    diagonal one, so Alg. 1 climbs one step per move and a walk started
    low on the staircase takes many rounds."""
    A = np.zeros((n, n))
    for j in range(n):
        A[j, j] = 2 * j + 1.0
        if j + 1 < n:
            A[j, j + 1] = 2 * j + 2.0
    return A


def test_rook_loop_runs_until_no_step_moves():
    """On the bidiagonal staircase the walks of Alg. 1 take tens of rounds;
    every rook pivot, in order, is the largest |residual| of its row and of
    its column (residuals from the direct CUR formula, numpy solve).  A walk
    cut after 8 rounds (a test option of the oracle) breaks that condition."""
    n = 64
    A = _bidiagonal(n)
    params = _matrix_as_sepsum(A)

    def rook_ok(o):
        _, _, rho, gam, _ = o.pivots(1)
        for z in range(len(rho)):
            I, J = list(rho[:z]), list(gam[:z])
            R = A.copy() if z == 0 else A - A[:, J] @ np.linalg.solve(A[np.ix_(I, J)], A[I, :])
            R[I, :] = 0.0
            R[:, J] = 0.0
            i, j = int(rho[z]), int(gam[z])
            if abs(R[i, j]) < np.abs(R[:, j]).max() or abs(R[i, j]) < np.abs(R[i, :]).max():
                return False
        return True

    for seed in (0, 2):
        o = Oracle([n, n], 1e-14, FN_SEPSUM, params, seed=seed, r_max=6, pivot="rook", grid=[1, 1])
        o.run()
        assert o.rook_rounds() > 8
        assert rook_ok(o)
        cut = Oracle([n, n], 1e-14, FN_SEPSUM, params, seed=seed, r_max=6, pivot="rook", grid=[1, 1], rook_iters=8)
        cut.run()
        assert not rook_ok(cut)
