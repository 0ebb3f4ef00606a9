"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle (oracle/stiles_oracle.c) is checked here against things that are
not itself: numpy/LAPACK factorizations and inverses, brute-force
determinants, closed forms, the paper's own 3 x 3 tile equations (Sec. III-A),
invariants, and the reported pivot failure.  A dropped term, a wrong sign or
index or a transposed operand anywhere in it breaks at least one of these.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sla

from paper_2504_19171_amd.inputs import arrowhead_spd

SHAPES = [
    # (nb, w, a, b)
    (40, 5, 3, 8),
    (37, 0, 3, 8),       # diagonal band + arrow
    (30, 5, 0, 8),       # no arrow
    (20, 19, 4, 8),      # dense band
    (50, 7, 6, 16),
    (13, 3, 2, 16),      # nb < b: one band tile
    (64, 9, 5, 16),
    (1, 0, 2, 4),
]


def dense_L(f):
    n = f.nb + f.a
    L = np.zeros((n, n))
    for i in range(f.nb):
        for t in range(f.w + 1):
            k = i - f.w + t
            if k >= 0:
                L[i, k] = f.Lr[i, t]
    if f.a:
        L[f.nb:, : f.nb] = f.LP
        L[f.nb:, f.nb:] = f.LC
    return L


def pattern_pairs(nb, a, w, b, oracle):
    """(i, j), i >= j, of the tile pattern of L."""
    out = []
    for j in range(nb):
        for i in range(j, oracle.selected_rows_last(nb, w, b, j) + 1):
            out.append((i, j))
        for r in range(a):
            out.append((nb + r, j))
    for c in range(a):
        for r in range(c, a):
            out.append((nb + r, nb + c))
    return out


def sigma_entry(S, nb, i, j):
    """Sigma[i, j] (i >= j) from the oracle's selected-inverse storage."""
    if i < nb:
        return S.Sb[i - j, j]
    if j < nb:
        return S.SP[i - nb, j]
    return S.SC[i - nb, j - nb]


@pytest.mark.parametrize("nb,w,a,b", SHAPES)
def test_cholesky_and_logdet_match_numpy(oracle_mod, nb, w, a, b):
    M = arrowhead_spd(nb, w, a, seed=11)
    A = M.dense()
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    assert f.info == 0
    np.testing.assert_allclose(dense_L(f), np.linalg.cholesky(A), rtol=0, atol=1e-13 * np.abs(A).max())
    sign, ld = np.linalg.slogdet(A)
    assert sign == 1.0
    assert abs(f.logdet - ld) <= 1e-13 * max(1.0, abs(ld))


@pytest.mark.parametrize("nb,w", [(60, 4), (33, 1), (25, 0), (40, 12)])
def test_band_cholesky_matches_lapack_pbtrf(oracle_mod, nb, w):
    """a = 0: the oracle's factor equals LAPACK's banded Cholesky (dpbtrf)."""
    M = arrowhead_spd(nb, w, 0, seed=5)
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    cb = sla.cholesky_banded(M.ab, lower=True)   # cb[d, j] = L[j+d, j]
    for d in range(w + 1):
        j = np.arange(nb - d)
        np.testing.assert_allclose(f.Lr[j + d, w - d], cb[d, : nb - d], rtol=1e-14, atol=1e-14)


def _leibniz_det(A):
    n = A.shape[0]
    tot = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for x in range(n) for y in range(x + 1, n) if perm[x] > perm[y])
        prod = 1.0
        for r in range(n):
            prod *= A[r, perm[r]]
        tot += (-1) ** inv * prod
    return tot


@pytest.mark.parametrize("nb,w,a", [(4, 1, 2), (5, 2, 1), (6, 0, 1), (3, 2, 3), (7, 3, 0)])
def test_logdet_brute_force(oracle_mod, nb, w, a):
    M = arrowhead_spd(nb, w, a, seed=2)
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    det = _leibniz_det(M.dense())
    assert det > 0
    assert abs(f.logdet - math.log(det)) <= 1e-12 * abs(math.log(det)) + 1e-13


def test_logdet_closed_forms(oracle_mod):
    # diagonal matrix: log det = sum log A_ii, Sigma = diag(1/A_ii)
    rng = np.random.default_rng(0)
    nb = 50
    ab = np.zeros((1, nb))
    ab[0] = rng.uniform(0.5, 3.0, nb)
    f = oracle_mod.cholesky(ab, np.zeros((0, nb)), np.zeros((0, 0)))
    assert abs(f.logdet - np.log(ab[0]).sum()) < 1e-12
    S = oracle_mod.selinv(f, 8)
    np.testing.assert_allclose(S.Sb[0], 1.0 / ab[0], rtol=1e-15)
    assert np.all(S.Sb[1:] == 0.0)
    # A = c I (with an arrow block that is also c I): log det = n log c
    c = 2.5
    nb, a = 30, 4
    ab = np.zeros((3, nb)); ab[0] = c
    P = np.zeros((a, nb)); C = c * np.eye(a)
    f = oracle_mod.cholesky(ab, P, C)
    assert abs(f.logdet - (nb + a) * math.log(c)) < 1e-12


@pytest.mark.parametrize("nb,w,a,b", SHAPES)
def test_selinv_matches_dense_inverse_on_pattern(oracle_mod, nb, w, a, b):
    M = arrowhead_spd(nb, w, a, seed=13)
    A = M.dense()
    Ai = np.linalg.inv(A)
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    S = oracle_mod.selinv(f, b)
    d = np.sqrt(np.diag(Ai))
    worst = 0.0
    for (i, j) in pattern_pairs(nb, a, w, b, oracle_mod):
        worst = max(worst, abs(sigma_entry(S, nb, i, j) - Ai[i, j]) / (d[i] * d[j]))
    assert worst < 1e-13
    # entries outside the tile pattern are left at zero
    for j in range(nb):
        last = oracle_mod.selected_rows_last(nb, w, b, j)
        assert np.all(S.Sb[last - j + 1:, j] == 0.0)
    # corner stored full symmetric
    if a:
        np.testing.assert_array_equal(S.SC, S.SC.T)


def test_selinv_row_identity(oracle_mod):
    """sum_k Sigma_ik A_ki = 1: A's pattern lies inside the selected pattern."""
    nb, w, a, b = 200, 11, 7, 16
    M = arrowhead_spd(nb, w, a, seed=21)
    A = M.dense()
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    S = oracle_mod.selinv(f, b)
    n = nb + a
    Sig = np.zeros((n, n))
    for (i, j) in pattern_pairs(nb, a, w, b, oracle_mod):
        Sig[i, j] = Sig[j, i] = sigma_entry(S, nb, i, j)
    rowsum = (Sig * A).sum(axis=1)   # A symmetric: sum_k Sigma_ik A_ki
    np.testing.assert_allclose(rowsum, 1.0, rtol=0, atol=1e-13)


def test_dense_case_matches_lapack_potri(oracle_mod):
    """w >= nb-1, a = 0: the pattern is the whole lower triangle; Sigma = dpotri."""
    nb, b = 24, 8
    M = arrowhead_spd(nb, nb - 1, 0, seed=4)
    A = M.dense()
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    S = oracle_mod.selinv(f, b)
    c, info = sla.lapack.dpotrf(A, lower=1)
    assert info == 0
    inv, info = sla.lapack.dpotri(c, lower=1)
    assert info == 0
    for j in range(nb):
        for i in range(j, nb):
            assert abs(S.Sb[i - j, j] - inv[i, j]) <= 1e-14 * math.sqrt(inv[i, i] * inv[j, j])


def test_paper_three_by_three_tile_equations(oracle_mod):
    """The tile relations printed in Sec. III-A for 3 x 3 tiles, evaluated
    literally, give the same Sigma as the oracle (dense matrix, tile t)."""
    t = 5
    nb = 3 * t
    M = arrowhead_spd(nb, nb - 1, 0, seed=9)
    A = M.dense()
    L = np.linalg.cholesky(A)
    Lb = lambda i, j: L[i * t:(i + 1) * t, j * t:(j + 1) * t]
    inv = np.linalg.inv
    S22 = inv(Lb(2, 2)).T @ inv(Lb(2, 2))
    S21 = -S22 @ Lb(2, 1) @ inv(Lb(1, 1))
    S11 = -inv(Lb(1, 1)).T @ Lb(2, 1).T @ S21 + inv(Lb(1, 1)).T @ inv(Lb(1, 1))
    S20 = -S21 @ Lb(1, 0) @ inv(Lb(0, 0)) - S22 @ Lb(2, 0) @ inv(Lb(0, 0))
    S12 = S21.T
    S10 = -S11 @ Lb(1, 0) @ inv(Lb(0, 0)) - S12 @ Lb(2, 0) @ inv(Lb(0, 0))
    S00 = -inv(Lb(0, 0)).T @ Lb(1, 0).T @ S10 - inv(Lb(0, 0)).T @ Lb(2, 0).T @ S20 \
        + inv(Lb(0, 0)).T @ inv(Lb(0, 0))
    blocks = {(2, 2): S22, (2, 1): S21, (1, 1): S11, (2, 0): S20, (1, 0): S10, (0, 0): S00}
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    S = oracle_mod.selinv(f, t)
    for (I, J), blk in blocks.items():
        for r in range(t):
            for c in range(t):
                i, j = I * t + r, J * t + c
                if i >= j:
                    assert abs(S.Sb[i - j, j] - blk[r, c]) < 1e-13 * math.sqrt(S.Sb[0, i] * S.Sb[0, j])
    # and the printed relations are A^{-1}
    np.testing.assert_allclose(np.block([[S00, S10.T, S20.T], [S10, S11, S21.T], [S20, S21, S22]]),
                               inv(A), rtol=1e-12, atol=1e-14)


def test_sigma_column_is_inverse_column(oracle_mod):
    nb, w, a = 80, 6, 5
    M = arrowhead_spd(nb, w, a, seed=1)
    Ai = np.linalg.inv(M.dense())
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    for j in (0, 17, nb - 1, nb, nb + a - 1):
        np.testing.assert_allclose(oracle_mod.sigma_column(f, j), Ai[:, j], rtol=0, atol=1e-15)


@pytest.mark.parametrize("col", [0, 9, 39, 41])
def test_not_positive_definite_reports_column(oracle_mod, col):
    nb, w, a = 40, 4, 3
    M = arrowhead_spd(nb, w, a, seed=3)
    if col < nb:
        M.ab[0, col] = -1.0
    else:
        M.C[col - nb, col - nb] = -1.0
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    assert f.info == col + 1
    assert math.isnan(f.logdet)


def test_scaling_invariance(oracle_mod):
    """A -> cA: Sigma -> Sigma / c, log det -> log det + n log c."""
    nb, w, a, b, c = 70, 5, 4, 16, 3.0
    M = arrowhead_spd(nb, w, a, seed=8)
    f1 = oracle_mod.cholesky(M.ab, M.P, M.C)
    f2 = oracle_mod.cholesky(c * M.ab, c * M.P, c * M.C)
    assert abs(f2.logdet - f1.logdet - (nb + a) * math.log(c)) < 1e-11
    S1, S2 = oracle_mod.selinv(f1, b), oracle_mod.selinv(f2, b)
    np.testing.assert_allclose(S2.Sb * c, S1.Sb, rtol=1e-13, atol=1e-17)
    np.testing.assert_allclose(S2.SP * c, S1.SP, rtol=1e-13, atol=1e-17)


def test_hadamard_and_diagonal_bounds(oracle_mod):
    """log det A <= sum log A_ii;  Sigma_ii >= 1 / A_ii;  |Sigma_ij| <= sqrt(Sigma_ii Sigma_jj)."""
    nb, w, a, b = 120, 9, 6, 16
    M = arrowhead_spd(nb, w, a, seed=31)
    A = M.dense()
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    assert f.logdet <= np.log(np.diag(A)).sum()
    S = oracle_mod.selinv(f, b)
    diagS = np.concatenate([S.Sb[0], np.diag(S.SC)])
    assert np.all(diagS >= 1.0 / np.diag(A) * (1 - 1e-14))
    for (i, j) in pattern_pairs(nb, a, w, b, oracle_mod):
        assert abs(sigma_entry(S, nb, i, j)) <= math.sqrt(diagS[i] * diagS[j]) * (1 + 1e-14)
