"""Pins for the CPU oracle: every check compares it with something other than
itself -- LAPACK (dense gesv, banded gbsv with pivoting), exact rational
arithmetic, closed forms, invariants of the factorisation and the paper's own
coefficient list.  A dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle fails at least one of these (the mutation
test in test_oracle_mutants.py demonstrates it)."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import Diagonals
from tests import _exact

U = np.finfo(np.float64).eps / 2


def random_dd(n, seed, symmetric=False, margin=1.5):
    """Random strictly diagonally dominant pentadiagonal (non-symmetric unless
    asked), diagonal of random sign."""
    g = np.random.Generator(np.random.PCG64(seed))
    a, b, d, e = (g.uniform(-1, 1, n) for _ in range(4))
    if symmetric:
        # row i: a_i = e_{i-2}, b_i = d_{i-1}
        a = np.concatenate([[0.0, 0.0], e[:-2]])
        b = np.concatenate([[0.0], d[:-1]])
    dg = [a.copy(), b.copy(), None, d.copy(), e.copy()]
    off = np.zeros(n)
    for i in range(n):
        for off_k, v in ((-2, a), (-1, b), (1, d), (2, e)):
            if 0 <= i + off_k < n:
                off[i] += abs(v[i])
    sign = 1.0 if symmetric else g.choice([-1.0, 1.0], n)
    c = sign * (margin * off + g.uniform(0.5, 1.0, n))
    dg[2] = c
    return Diagonals(*dg)


def kappa1(dg):
    return np.linalg.cond(oracle.dense(dg), 1)


def relerr(x, ref):
    return np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300)


# ---------------------------------------------------------------- paper values
def test_assemble_matches_paper_coefficients():
    """Sec. 2.3: a = e = sigma, b = d = -4 sigma, c = 1 + 6 sigma (golden file)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_coefficients.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for sig_s, a_s, b_s, c_s, d_s, e_s in rows:
        sigma = float(sig_s)
        n = 9
        dg = oracle.assemble_d4(n, sigma)
        i = 4  # an interior row
        assert (dg.a[i], dg.b[i], dg.c[i], dg.d[i], dg.e[i]) == tuple(
            float(v) for v in (a_s, b_s, c_s, d_s, e_s))
        # truncated boundary rows: out-of-range entries dropped
        assert dg.a[0] == dg.a[1] == dg.b[0] == 0.0
        assert dg.d[n - 1] == dg.e[n - 2] == dg.e[n - 1] == 0.0


# ------------------------------------------------------------- LAPACK pins
@pytest.mark.parametrize("n", list(range(1, 33)))
def test_dense_gesv_nonsymmetric(n):
    dg = random_dd(n, seed=100 + n)
    A = oracle.dense(dg)
    g = np.random.Generator(np.random.PCG64(7 + n))
    F = g.uniform(-1, 1, (n, 5))
    X = oracle.solve(dg, F)
    ref = np.linalg.solve(A, F)
    assert relerr(X, ref) <= 64 * U * kappa1(dg)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 17, 32])
@pytest.mark.parametrize("sigma", [0.1, 1.0, 50.0, 200.0, 1e4])
def test_dense_gesv_d4(n, sigma):
    dg = oracle.assemble_d4(n, sigma)
    F = np.random.Generator(np.random.PCG64(n)).uniform(-1, 1, (n, 3))
    X = oracle.solve(dg, F)
    ref = np.linalg.solve(oracle.dense(dg), F)
    assert relerr(X, ref) <= 64 * U * kappa1(dg)


def _banded(dg):
    n = dg.n
    ab = np.zeros((5, n))
    for i in range(n):
        for off, v in ((-2, dg.a), (-1, dg.b), (0, dg.c), (1, dg.d), (2, dg.e)):
            k = i + off
            if 0 <= k < n:
                ab[2 + i - k, k] = v[i]
    return ab


@pytest.mark.parametrize("n", [100, 1000, 4096])
@pytest.mark.parametrize("sigma", [0.1, 1.0, 50.0, 200.0, 1e4])
def test_gbsv_d4(n, sigma):
    """LAPACK banded solve with partial pivoting (a different algorithm)."""
    dg = oracle.assemble_d4(n, sigma)
    F = np.random.Generator(np.random.PCG64(n + 3)).uniform(-1, 1, (n, 4))
    X = oracle.solve(dg, F)
    ref = scipy.linalg.solve_banded((2, 2), _banded(dg), F)
    assert relerr(X, ref) <= 64 * U * (1 + 16 * sigma)


@pytest.mark.parametrize("n", [50, 777])
def test_gbsv_nonsymmetric(n):
    dg = random_dd(n, seed=n)
    F = np.random.Generator(np.random.PCG64(n)).uniform(-1, 1, (n, 3))
    X = oracle.solve(dg, F)
    ref = scipy.linalg.solve_banded((2, 2), _banded(dg), F)
    assert relerr(X, ref) <= 1e-13


# --------------------------------------------------------------- exact rationals
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 12])
def test_exact_rational_d4(n):
    sigma = Fraction(3, 2)
    dg = oracle.assemble_d4(n, float(sigma))
    A = _exact.dense_from_diagonals(*dg)
    f = [Fraction(((7 * i) % 11) - 5, 3) for i in range(n)]
    x = _exact.solve(A, f)
    X = oracle.solve(dg, np.array([float(v) for v in f]))
    ref = np.array([float(v) for v in x])
    assert relerr(X, ref) <= 16 * U * (1 + 16 * float(sigma))


@pytest.mark.parametrize("n", [3, 6, 11])
def test_exact_rational_nonsymmetric(n):
    g = np.random.Generator(np.random.PCG64(n))
    ints = lambda: g.integers(-4, 5, n).astype(np.float64)
    a, b, d, e = ints(), ints(), ints(), ints()
    c = 20.0 + g.integers(0, 5, n)
    dg = Diagonals(a, b, c, d, e)
    A = _exact.dense_from_diagonals(*dg)
    f = [Fraction(int(v)) for v in g.integers(-9, 10, n)]
    x = _exact.solve(A, f)
    X = oracle.solve(dg, np.array([float(v) for v in f]))
    assert relerr(X, np.array([float(v) for v in x])) <= 64 * U * kappa1(dg)


# ------------------------------------------------------------------ closed forms
def test_sigma_zero_is_identity_bitwise():
    n = 37
    dg = oracle.assemble_d4(n, 0.0)
    fac = oracle.factor(dg)
    assert np.all(fac.alpha == 1.0)
    assert np.all(fac.beta == 0.0) and np.all(fac.gamma == 0.0) and np.all(fac.delta == 0.0)
    F = np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, (n, 9))
    assert np.array_equal(oracle.solve(dg, F, fac), F)


@pytest.mark.parametrize("sigma,k", [(7.0, 5), (0.3, 1), (123.0, 40)])
def test_sine_modes_of_i_plus_sigma_t2(sigma, k):
    """I + sigma*T^2, T = tridiag(-1, 2, -1): the Dirichlet sine modes
    s_k(j) = sin(pi k j/(n+1)) are eigenvectors with eigenvalue
    1 + sigma*mu_k^2, mu_k = 2 - 2 cos(pi k/(n+1))."""
    n = 100
    dg = oracle.assemble_d4(n, sigma)
    dg.c[0] = dg.c[n - 1] = 1.0 + 5.0 * sigma     # T^2 has 5 in its corners
    j = np.arange(1, n + 1)
    s = np.sin(np.pi * k * j / (n + 1))
    mu = 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
    X = oracle.solve(dg, s)
    assert relerr(X, s / (1.0 + sigma * mu * mu)) <= 64 * U * (1 + 16 * sigma)


# ------------------------------------------------------------ factor invariants
@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 64])
def test_factors_reproduce_matrix(n):
    """L R == A entrywise (the definition of the factorisation)."""
    for dg in (random_dd(n, seed=3 * n), oracle.assemble_d4(n, 50.0)):
        fac = oracle.factor(dg)
        L = np.zeros((n, n))
        R = np.eye(n)
        for i in range(n):
            L[i, i] = fac.alpha[i]
            if i >= 1:
                L[i, i - 1] = fac.beta[i]
                R[i - 1, i] = fac.gamma[i - 1]
            if i >= 2:
                L[i, i - 2] = dg.a[i]
                R[i - 2, i] = fac.delta[i - 2]
        A = oracle.dense(dg)
        assert np.max(np.abs(L @ R - A)) <= 16 * U * np.max(np.abs(A))


@pytest.mark.parametrize("sigma", [0.1, 1.0, 50.0, 200.0, 1e4])
def test_factor_invariants_spd(sigma):
    n = 300
    dg = oracle.assemble_d4(n, sigma)
    fac = oracle.factor(dg)
    assert np.all(fac.alpha > 0)                            # SPD => positive pivots
    # symmetric A = R^T diag(alpha) R  =>  beta_i = alpha_{i-1} gamma_{i-1},
    # a_i = alpha_{i-2} delta_{i-2}
    assert np.allclose(fac.beta[1:], fac.alpha[:-1] * fac.gamma[:-1], rtol=8 * U, atol=0)
    assert np.allclose(dg.a[2:], fac.alpha[:-2] * fac.delta[:-2], rtol=8 * U, atol=0)
    sign, logdet = np.linalg.slogdet(oracle.dense(dg))
    assert sign == 1.0
    assert abs(np.sum(np.log(fac.alpha)) - logdet) <= 1e-12 * abs(logdet) + 1e-12


@pytest.mark.parametrize("sigma", [0.1, 1.0, 50.0, 200.0, 1e4])
def test_factor_interior_limit(sigma):
    """Away from the boundary the factors of I + sigma*D4 converge to the
    spectral factor of the symbol 1 + sigma (2 - z - 1/z)^2: with z1 the root
    of z + 1/z = 2 - i/sqrt(sigma) of modulus > 1, delta -> 1/|z1|^2,
    gamma -> -2 Re(1/z1), alpha -> sigma |z1|^2."""
    n = 1200
    fac = oracle.factor(oracle.assemble_d4(n, sigma))
    c = 2.0 - 1j / math.sqrt(sigma)
    r = np.roots([1.0, -c, 1.0])
    z1 = r[np.argmax(np.abs(r))]
    i = n // 2
    assert abs(fac.delta[i] * abs(z1) ** 2 - 1) < 1e-12
    assert abs(fac.gamma[i] / (-2 * (1 / z1).real) - 1) < 1e-12
    assert abs(fac.alpha[i] / (sigma * abs(z1) ** 2) - 1) < 1e-12


# ------------------------------------------------------- manufactured solutions
@pytest.mark.parametrize("k", [-3, 0, 5])
def test_manufactured_dyadic_exact_rhs(k):
    """sigma = 2^k and small integer x*: f = A x* is exact in FP64, so the
    compensated residual of x* is exactly zero and the solve recovers x*."""
    n = 513
    sigma = 2.0 ** k
    dg = oracle.assemble_d4(n, sigma)
    xs = np.random.Generator(np.random.PCG64(11)).integers(-1000, 1001, (n, 3)).astype(float)
    F = oracle.matvec(dg, xs)
    eta, rho = oracle.residual(dg, xs, F)
    assert np.all(eta == 0.0) and np.all(rho == 0.0)
    X = oracle.solve(dg, F)
    assert relerr(X, xs) <= 64 * U * (1 + 16 * sigma)


def test_manufactured_seeded_longdouble():
    n = 2048
    sigma = 200.0
    dg = oracle.assemble_d4(n, sigma)
    xs = np.random.Generator(np.random.PCG64(12)).uniform(-1, 1, (n, 4))
    A = [np.asarray(v, dtype=np.longdouble) for v in dg]
    xl = xs.astype(np.longdouble)
    F = A[2][:, None] * xl
    F[2:] += A[0][2:, None] * xl[:-2]
    F[1:] += A[1][1:, None] * xl[:-1]
    F[:-1] += A[3][:-1, None] * xl[1:]
    F[:-2] += A[4][:-2, None] * xl[2:]
    X = oracle.solve(dg, F.astype(np.float64))
    assert relerr(X, xs) <= 64 * U * (1 + 16 * sigma)


# ------------------------------------------------------------------ zero pivots
def test_zero_pivot_first_row():
    dg = oracle.assemble_d4(6, 1.0)
    dg.c[0] = 0.0
    with pytest.raises(oracle.ZeroPivot) as ei:
        oracle.factor(dg)
    assert ei.value.row == 0


def test_zero_pivot_singular_leading_block():
    """[[1, 1], [1, 1]] leading block: alpha_2 = 1 - 1*1 = 0."""
    dg = Diagonals(np.zeros(2), np.array([0.0, 1.0]), np.array([1.0, 1.0]),
                   np.array([1.0, 0.0]), np.zeros(2))
    with pytest.raises(oracle.ZeroPivot) as ei:
        oracle.factor(dg)
    assert ei.value.row == 1


def test_non_finite_pivot():
    dg = oracle.assemble_d4(8, 1.0)
    dg.c[5] = np.nan
    with pytest.raises(oracle.ZeroPivot) as ei:
        oracle.factor(dg)
    assert ei.value.row == 5


def test_unused_entries_ignored():
    n = 10
    dg = oracle.assemble_d4(n, 3.0)
    junk = Diagonals(*(v.copy() for v in dg))
    junk.a[0] = junk.a[1] = junk.b[0] = 99.0
    junk.d[n - 1] = junk.e[n - 2] = junk.e[n - 1] = -77.0
    F = np.random.Generator(np.random.PCG64(2)).uniform(-1, 1, (n, 3))
    assert np.array_equal(oracle.solve(dg, F), oracle.solve(junk, F))
    assert all(np.array_equal(x, y) for x, y in zip(oracle.factor(dg), oracle.factor(junk)))


# ---------------------------------------------------------------- batch semantics
def test_columns_independent_and_permutation_equivariant():
    n, m = 300, 70
    dg = oracle.assemble_d4(n, 50.0)
    F = np.random.Generator(np.random.PCG64(5)).uniform(-1, 1, (n, m))
    X = oracle.solve(dg, F)
    for j in (0, 33, m - 1):
        assert np.array_equal(X[:, j], oracle.solve(dg, F[:, j]))
    perm = np.random.Generator(np.random.PCG64(6)).permutation(m)
    assert np.array_equal(oracle.solve(dg, F[:, perm]), X[:, perm])


def test_linearity():
    n = 400
    dg = oracle.assemble_d4(n, 1e4)
    g = np.random.Generator(np.random.PCG64(8))
    f1, f2 = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    lhs = oracle.solve(dg, 2.0 * f1 - 0.5 * f2)
    rhs = 2.0 * oracle.solve(dg, f1) - 0.5 * oracle.solve(dg, f2)
    assert relerr(lhs, rhs) <= 64 * U * (1 + 16e4)


def test_ld_larger_than_batch():
    n, m, ld = 50, 7, 13
    dg = oracle.assemble_d4(n, 2.0)
    g = np.random.Generator(np.random.PCG64(9))
    big = g.uniform(-1, 1, (n, ld))
    ref = oracle.solve(dg, big[:, :m])
    fac = oracle.factor(dg)
    view = big[:, :m]
    pad = big[:, m:].copy()
    oracle.solve_inplace(dg, fac, view)
    assert np.array_equal(big[:, :m], ref)
    assert np.array_equal(big[:, m:], pad)       # padding columns untouched


# ---------------------------------------------------------- residual evaluator
def test_residual_matches_exact_rational():
    n = 9
    dg = random_dd(n, seed=4)
    g = np.random.Generator(np.random.PCG64(4))
    x = g.uniform(-1, 1, n)
    f = g.uniform(-1, 1, n)
    A = _exact.dense_from_diagonals(*dg)
    Ax = _exact.matvec(A, list(x))
    r = np.array([float(Fraction(f[i]) - Ax[i]) for i in range(n)])
    eta, rho = oracle.residual(dg, x, f)
    anorm = np.max(np.sum(np.abs(oracle.dense(dg)), axis=1))
    assert eta[0] == pytest.approx(np.max(np.abs(r)) / (anorm * np.max(np.abs(x)) + np.max(np.abs(f))),
                                   rel=1e-14)
    assert rho[0] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(f), rel=1e-14)


@pytest.mark.parametrize("sigma", [0.1, 50.0, 1e4])
def test_backward_error_of_oracle_solution_is_small(sigma):
    n = 4096
    dg = oracle.assemble_d4(n, sigma)
    F = np.random.Generator(np.random.PCG64(10)).uniform(-1, 1, (n, 8))
    X = oracle.solve(dg, F)
    eta, rho = oracle.residual(dg, X, F)
    assert np.all(eta <= 1e-15)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_backward_error_of_non_finite_solution_is_not_finite(bad):
    """A solution with a NaN or an infinite entry has no finite backward
    error: eta must come out non-finite, never 0 (a max that skipped the NaN
    would report a clean column)."""
    n = 12
    dg = oracle.assemble_d4(n, 2.0)
    F = np.random.Generator(np.random.PCG64(11)).uniform(-1, 1, (n, 3))
    X = oracle.solve(dg, F)
    X[5, 1] = bad
    X[:, 2] = bad
    eta, _ = oracle.residual(dg, X, F)
    assert np.isfinite(eta[0]) and eta[0] <= 1e-15
    assert not np.isfinite(eta[1])
    assert not np.isfinite(eta[2])
