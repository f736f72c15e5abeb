"""Exact rational reference (test pin, independent of the oracle): dense
Gaussian elimination over fractions.Fraction with partial pivoting on the
first non-zero entry.  Only for tiny systems."""
from fractions import Fraction


def dense_from_diagonals(a, b, c, d, e):
    n = len(c)
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for off, v in ((-2, a), (-1, b), (0, c), (1, d), (2, e)):
            k = i + off
            if 0 <= k < n:
                A[i][k] = Fraction(v[i])
    return A


def solve(A, f):
    n = len(A)
    M = [list(map(Fraction, row)) + [Fraction(f[i])] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(col + 1, n):
            if M[r][col] != 0:
                m = M[r][col] / M[col][col]
                for k in range(col, n + 1):
                    M[r][k] -= m * M[col][k]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n] - sum(M[i][k] * x[k] for k in range(i + 1, n))
        x[i] = s / M[i][i]
    return x


def matvec(A, x):
    return [sum(A[i][k] * Fraction(x[k]) for k in range(len(x))) for i in range(len(A))]
