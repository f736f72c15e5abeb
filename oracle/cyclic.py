"""Cyclic (periodic) pentadiagonal solve and the Crank-Nicolson hyperdiffusion
validation -- TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

Sec. 2.3: the periodic hyperdiffusion matrix A has entries wrapping round the
corners.  Navon's bordering removes the last two rows and columns: E is the
leading (N-2) x (N-2) block (an ordinary pentadiagonal matrix), k the last two
columns without their last two rows, h^T the last two rows without their last
two columns, C2 the trailing 2 x 2 block.  Then
    (x_{N-1}, x_N) = [C2 - h^T E^{-1} k]^{-1} [(f_{N-1}, f_N) - h^T E^{-1} f^]
    X^            = E^{-1} [f^ - k (x_{N-1}, x_N)]
with [C2 - h^T E^{-1} k]^{-1} and h^T E^{-1} computed once (the paper
precomputes both).  The solves with E are the oracle's FP64 pentadiagonal
solve (Sec. 2.4).

Row-indexed cyclic diagonals: row i holds a[i] at column (i-2) mod N,
b[i] at (i-1) mod N, c[i] at i, d[i] at (i+1) mod N, e[i] at (i+2) mod N;
N >= 5 so that no two entries of a row share a column.
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np

from . import Diagonals, factor, solve_inplace


def cyclic_d4(n: int, sigma: float) -> Diagonals:
    """The periodic matrix of Sec. 2.3: a = e = sigma, b = d = -4 sigma,
    c = 1 + 6 sigma in every row, corners included."""
    if n < 5:
        raise ValueError("cyclic matrices need n >= 5")
    f = lambda v: np.full(n, v, dtype=np.float64)
    return Diagonals(f(sigma), f(-4.0 * sigma), f(1.0 + 6.0 * sigma), f(-4.0 * sigma), f(sigma))


def dense_cyclic(dg: Diagonals) -> np.ndarray:
    n = dg.n
    A = np.zeros((n, n))
    for i in range(n):
        for off, v in ((-2, dg.a), (-1, dg.b), (0, dg.c), (1, dg.d), (2, dg.e)):
            A[i, (i + off) % n] += v[i]
    return A


class Bordering(NamedTuple):
    E: Diagonals          # leading (N-2) x (N-2) block, truncated pentadiagonal
    Efac: object          # its A = LR factors
    k: np.ndarray         # (N-2, 2)
    hT: np.ndarray        # (2, N-2)
    C2: np.ndarray        # (2, 2)
    hTEinv: np.ndarray    # (2, N-2) = h^T E^{-1}
    Minv: np.ndarray      # [C2 - h^T E^{-1} k]^{-1}


def bordering(dg: Diagonals) -> Bordering:
    """Precomputation of Sec. 2.3 (eq. first_two): E, h, k, C2 from the
    cyclic matrix, then h^T E^{-1} and [C2 - h^T E^{-1} k]^{-1}."""
    n = dg.n
    if n < 5:
        raise ValueError("cyclic matrices need n >= 5")
    A = dense_cyclic(dg)
    m = n - 2
    E = Diagonals(*(np.array(v[:m]) for v in dg))
    Efac = factor(E)
    k = A[:m, m:].copy()
    hT = A[m:, :m].copy()
    C2 = A[m:, m:].copy()
    # h^T E^{-1} = (E^{-T} h)^T: solve E^T w = h through dense E (small
    # matrices only need this once); the oracle keeps it plain.
    Ed = A[:m, :m]
    hTEinv = np.linalg.solve(Ed.T, hT.T).T
    Minv = np.linalg.inv(C2 - hTEinv @ k)
    return Bordering(E, Efac, k, hT, C2, hTEinv, Minv)


def solve_cyclic(bd: Bordering, F: np.ndarray) -> np.ndarray:
    """x = A^{-1} F for the cyclic matrix, F of shape (n,) or (n, batch),
    in the paper's order: the last two unknowns first (eq. first_two), then
    the rest by a pentadiagonal solve with E (eq. solve)."""
    F = np.asarray(F, dtype=np.float64)
    one = F.ndim == 1
    F2 = F.reshape(F.shape[0], -1)
    m = F2.shape[0] - 2
    fhat, ftail = F2[:m], F2[m:]
    xt = bd.Minv @ (ftail - bd.hTEinv @ fhat)
    X = np.array(fhat - bd.k @ xt, order="C")
    solve_inplace(bd.E, bd.Efac, X)
    out = np.vstack([X, xt])
    return out[:, 0] if one else out


def cn_rhs(C: np.ndarray, sigma: float) -> np.ndarray:
    """Explicit half of the Crank-Nicolson step (Sec. 2.3, the f_i of the
    matrix system): f_i = -s C_{i-2} + 4s C_{i-1} + (1 - 6s) C_i
    + 4s C_{i+1} - s C_{i+2}, indices periodic, along axis 0."""
    C = np.asarray(C, dtype=np.float64)
    r = lambda k: np.roll(C, k, axis=0)   # r(k)[i] = C[i-k]
    return (-sigma * r(2) + 4.0 * sigma * r(1) + (1.0 - 6.0 * sigma) * C
            + 4.0 * sigma * r(-1) - sigma * r(-2))


def cn_run(sigma: float, C0: np.ndarray, steps: int) -> np.ndarray:
    """`steps` Crank-Nicolson steps of the periodic hyperdiffusion scheme
    (Sec. 2.3) from C0 of shape (n,) or (n, batch): each step solves
    A C^{k+1} = (2I - A) C^k with the bordering solve."""
    C = np.asarray(C0, dtype=np.float64)
    bd = bordering(cyclic_d4(C.shape[0], sigma))
    for _ in range(int(steps)):
        C = solve_cyclic(bd, cn_rhs(C, sigma))
    return C


def hyperdiffusion_cn(n: int, dt: float, T: float, mode: int = 2):
    """Sec. 2.5 validation run: dC/dt = -d^4C/dx^4 on [0, 1) periodic,
    C(x, 0) = cos(2 pi mode x), Crank-Nicolson with sigma = dt / (2 dx^4),
    dx = 1/n, grid x_i = i dx (i = 1..n).  Returns (C(T), exact(T), eps_N)
    with eps_N the RMS error of eq. myerr."""
    dx = 1.0 / n
    sigma = dt / (2.0 * dx ** 4)
    x = dx * np.arange(1, n + 1)
    kw = 2.0 * np.pi * mode
    steps = int(round(T / dt))
    C = cn_run(sigma, np.cos(kw * x), steps)
    exact = np.exp(-kw ** 4 * steps * dt) * np.cos(kw * x)
    eps = float(np.sqrt(np.mean((C - exact) ** 2)))
    return C, exact, eps
