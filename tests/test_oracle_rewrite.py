"""Pins for the oracle's per-system refactor-and-solve (every system with its
own matrix, factored on every call; the paper's refactor-every-step mode,
Sec. 3), against dense LAPACK solves and exact invariants."""
import numpy as np
import pytest

import oracle

U = np.finfo(np.float64).eps / 2


def per_system(n, m, seed, dominance=1.5):
    """Row-indexed diagonals of shape (n, m), one non-symmetric diagonally
    dominant matrix per column, entries outside each matrix zeroed."""
    g = np.random.Generator(np.random.PCG64(seed))
    a, b, d, e = (g.uniform(-1, 1, (n, m)) for _ in range(4))
    a[:2] = 0.0
    b[:1] = 0.0
    d[n - 1:] = 0.0
    e[max(n - 2, 0):] = 0.0
    c = (dominance * (np.abs(a) + np.abs(b) + np.abs(d) + np.abs(e)) + g.uniform(0.5, 1.0, (n, m))) \
        * g.choice([-1.0, 1.0], (n, m))
    return a, b, c, d, e


def dense_of(diags, j):
    return oracle.dense(oracle.Diagonals(*(np.ascontiguousarray(x[:, j]) for x in diags)))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 13, 32])
def test_rewrite_matches_dense_per_system(n):
    m = 6
    diags = per_system(n, m, seed=n)
    F = np.random.Generator(np.random.PCG64(n + 50)).uniform(-1, 1, (n, m))
    X = oracle.rewrite_solve(*diags, F)
    for j in range(m):
        A = dense_of(diags, j)
        ref = np.linalg.solve(A, F[:, j])
        kappa = np.linalg.cond(A, np.inf)
        assert np.max(np.abs(X[:, j] - ref)) <= 64 * U * kappa * np.max(np.abs(ref))


def test_rewrite_residual_small():
    n, m = 200, 9
    diags = per_system(n, m, seed=3)
    F = np.random.Generator(np.random.PCG64(4)).uniform(-1, 1, (n, m))
    X = oracle.rewrite_solve(*diags, F)
    for j in range(m):
        r = dense_of(diags, j) @ X[:, j] - F[:, j]
        assert np.max(np.abs(r)) <= 1e-13


def test_rewrite_column_permutation_equivariant():
    n, m = 40, 7
    diags = per_system(n, m, seed=5)
    F = np.random.Generator(np.random.PCG64(6)).uniform(-1, 1, (n, m))
    X = oracle.rewrite_solve(*diags, F)
    perm = np.random.Generator(np.random.PCG64(7)).permutation(m)
    Xp = oracle.rewrite_solve(*(x[:, perm] for x in diags), F[:, perm])
    assert np.array_equal(Xp, X[:, perm])


def test_rewrite_each_column_its_own_sigma():
    """Systems I + sigma_j D4 with different sigma_j: column j is the solve of
    its own matrix (Sec. 2.3 coefficients), checked densely."""
    n = 24
    sig = np.array([0.0, 0.1, 5.0, 200.0])
    cols = [oracle.assemble_d4(n, s) for s in sig]
    diags = [np.stack([getattr(dg, k) for dg in cols], axis=1) for k in "abcde"]
    F = np.random.Generator(np.random.PCG64(8)).uniform(-1, 1, (n, len(sig)))
    X = oracle.rewrite_solve(*diags, F)
    for j, s in enumerate(sig):
        A = oracle.dense(cols[j])
        ref = np.linalg.solve(A, F[:, j])
        assert np.max(np.abs(X[:, j] - ref)) <= 64 * U * (1 + 16 * s) * np.max(np.abs(ref))
    assert np.array_equal(X[:, 0], F[:, 0])   # sigma = 0: the identity


def test_rewrite_reports_system_and_row_of_zero_pivot():
    """The first system (lowest index) whose factorisation meets a zero pivot
    is reported with that row.  System 1: c_0 = 1, d_0 = 2, b_1 = 3, c_1 = 6
    gives alpha_1 = 6 - 3 * 2 = 0 exactly; system 3: c_0 = 0."""
    n, m = 10, 5
    a, b, c, d, e = (x.copy() for x in per_system(n, m, seed=9))
    c[0, 1], d[0, 1], b[1, 1], c[1, 1] = 1.0, 2.0, 3.0, 6.0
    c[0, 3] = 0.0
    F = np.ones((n, m))
    with pytest.raises(oracle.SystemZeroPivot) as ei:
        oracle.rewrite_solve(a, b, c, d, e, F)
    assert (ei.value.system, ei.value.row) == (1, 1)
    c[:, 1] = per_system(n, m, seed=9)[2][:, 1]
    with pytest.raises(oracle.SystemZeroPivot) as ei:
        oracle.rewrite_solve(a, b, c, d, e, F)
    assert (ei.value.system, ei.value.row) == (3, 0)
