"""CPU oracle for the batched pentadiagonal solve -- TEST INFRASTRUCTURE ONLY.

Plain FP64 reference implementation of Gloster, O Naraigh and Pang,
"cuPentBatch -- A batched pentadiagonal solver for NVIDIA GPUs"
(arXiv:1807.07382).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_1807_07382_amd``) and neither imports the other;
the product must never fall back to it.

The arithmetic lives in ``pent_oracle.c`` (compiled with gcc, IEEE FP64, no
contraction); this module only marshals numpy arrays into it, plus the plain
numpy workload drivers in :mod:`oracle.workloads`.

Layout: right-hand sides are 2-D arrays of shape (n, batch) -- row i is the
i-th unknown of every system, which is the interleaved, batch-fastest layout
of the paper's GPU implementation (Sec. 2.6).  Rows are 0-based.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pent_oracle.c")
# PENT_ORACLE_LIB names another build of the same source (the sanitizer job's)
_LIB_PATH = os.environ.get("PENT_ORACLE_LIB") or os.path.join(_HERE, "_pent_oracle.so")
_lib = None

OK, INVALID, ZERO_PIVOT = 0, 1, 2

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle's C source into ``oracle/_pent_oracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_assemble_d4.argtypes = [I64, ctypes.c_double, P, P, P, P, P]
        lib.orc_factor.argtypes = [I64, P, P, P, P, P, P, P, P, P, ctypes.POINTER(I64)]
        lib.orc_solve.argtypes = [I64, P, P, P, P, P, P, I64, I64]
        lib.orc_residual.argtypes = [I64, P, P, P, P, P, P, I64, P, I64, I64, P, P]
        lib.orc_matvec.argtypes = [I64, P, P, P, P, P, P, I64, P, I64, I64]
        for f in (lib.orc_assemble_d4, lib.orc_factor, lib.orc_solve, lib.orc_residual,
                  lib.orc_matvec, lib.orc_num_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(x: np.ndarray):
    return x.ctypes.data_as(ctypes.c_void_p)


def _vec(x, n):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.shape != (n,):
        raise ValueError(f"diagonal must have shape ({n},), got {x.shape}")
    return x


class Diagonals(NamedTuple):
    """Row-indexed diagonals (Sec. 2.4): row i holds a (col i-2), b (i-1),
    c (i), d (i+1), e (i+2)."""
    a: np.ndarray
    b: np.ndarray
    c: np.ndarray
    d: np.ndarray
    e: np.ndarray

    @property
    def n(self) -> int:
        return int(self.c.shape[0])


class Factors(NamedTuple):
    """A = L R (Sec. 2.4): alpha, beta, epsilon(=a) form L; gamma, delta form R."""
    alpha: np.ndarray
    beta: np.ndarray
    gamma: np.ndarray
    delta: np.ndarray


class ZeroPivot(ArithmeticError):
    def __init__(self, row: int):
        super().__init__(f"zero or non-finite pivot alpha at row {row}")
        self.row = row


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_num_threads())


def assemble_d4(n: int, sigma: float) -> Diagonals:
    """I + sigma*D4 with the five-point fourth-difference row
    (sigma, -4 sigma, 1 + 6 sigma, -4 sigma, sigma) of Sec. 2.3, with the
    entries outside the matrix dropped (non-periodic, truncated)."""
    arrs = [np.empty(n, dtype=np.float64) for _ in range(5)]
    rc = _load().orc_assemble_d4(int(n), float(sigma), *[_p(x) for x in arrs])
    if rc != OK:
        raise ValueError("invalid arguments to assemble_d4")
    return Diagonals(*arrs)


def factor(diags: Diagonals) -> Factors:
    """A = L R without pivoting (Sec. 2.4).  Raises ZeroPivot(row)."""
    n = diags.n
    dg = [_vec(x, n) for x in diags]
    out = [np.zeros(n, dtype=np.float64) for _ in range(4)]
    bad = ctypes.c_int64(-1)
    rc = _load().orc_factor(n, *[_p(x) for x in dg], *[_p(x) for x in out], ctypes.byref(bad))
    if rc == ZERO_PIVOT:
        raise ZeroPivot(int(bad.value))
    if rc != OK:
        raise ValueError("invalid arguments to factor")
    return Factors(*out)


def _check_F(F: np.ndarray, n: int):
    if F.dtype != np.float64 or F.ndim != 2 or F.shape[0] != n:
        raise ValueError(f"F must be float64 of shape ({n}, batch), got {F.dtype} {F.shape}")
    if F.shape[1] == 0:
        return 0
    if (F.shape[1] > 1 and F.strides[1] != 8) or F.strides[0] % 8:
        raise ValueError("F must have unit stride along the batch axis")
    return F.strides[0] // 8


def solve_inplace(diags: Diagonals, fac: Factors, F: np.ndarray) -> np.ndarray:
    """Overwrite F (shape (n, batch), batch-fastest) with the solutions."""
    n = diags.n
    ld = _check_F(F, n)
    a = _vec(diags.a, n)
    fs = [_vec(x, n) for x in fac]
    rc = _load().orc_solve(n, _p(a), *[_p(x) for x in fs], _p(F), F.shape[1], ld)
    if rc != OK:
        raise ValueError("invalid arguments to solve")
    return F


def solve(diags: Diagonals, F: np.ndarray, fac: Factors | None = None) -> np.ndarray:
    """Return A^{-1} F (a new array); F has shape (n,) or (n, batch)."""
    F = np.asarray(F, dtype=np.float64)
    one = F.ndim == 1
    X = np.array(F.reshape(F.shape[0], -1), dtype=np.float64, order="C", copy=True)
    if fac is None:
        fac = factor(diags)
    solve_inplace(diags, fac, X)
    return X[:, 0] if one else X


def residual(diags: Diagonals, X: np.ndarray, F: np.ndarray):
    """Per-column backward error eta = ||r||_inf/(||A||_inf ||x||_inf + ||f||_inf)
    and relative residual rho = ||r||_2/||f||_2 with r = f - A x evaluated in
    compensated (Dot2) arithmetic."""
    n = diags.n
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
        F = F[:, None]
    X = np.ascontiguousarray(X)
    F = np.ascontiguousarray(F)
    if X.shape != F.shape or X.shape[0] != n:
        raise ValueError("X and F must both have shape (n, batch)")
    dg = [_vec(x, n) for x in diags]
    m = X.shape[1]
    eta = np.zeros(m)
    rho = np.zeros(m)
    rc = _load().orc_residual(n, *[_p(x) for x in dg], _p(X), m, _p(F), m, m, _p(eta), _p(rho))
    if rc != OK:
        raise ValueError("invalid arguments to residual")
    return eta, rho


def matvec(diags: Diagonals, X: np.ndarray) -> np.ndarray:
    """Plain FP64 banded product A X."""
    n = diags.n
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    one = X.ndim == 1
    X2 = X.reshape(n, -1)
    Y = np.empty_like(X2)
    dg = [_vec(x, n) for x in diags]
    rc = _load().orc_matvec(n, *[_p(x) for x in dg], _p(X2), X2.shape[1], _p(Y), Y.shape[1],
                            X2.shape[1])
    if rc != OK:
        raise ValueError("invalid arguments to matvec")
    return Y[:, 0] if one else Y


def dense(diags: Diagonals) -> np.ndarray:
    """The n x n matrix the row-indexed diagonals describe (for small tests)."""
    n = diags.n
    A = np.zeros((n, n))
    for i in range(n):
        for off, v in ((-2, diags.a), (-1, diags.b), (0, diags.c), (1, diags.d), (2, diags.e)):
            k = i + off
            if 0 <= k < n:
                A[i, k] = v[i]
    return A


class SystemZeroPivot(ArithmeticError):
    """Factorisation of one system's own matrix stopped (system j, row i)."""

    def __init__(self, system: int, row: int):
        super().__init__(f"system {system}: zero or non-finite pivot at row {row}")
        self.system = system
        self.row = row


def rewrite_solve(a, b, c, d, e, F) -> np.ndarray:
    """Every system with its own matrix, factored and solved in one call
    (the paper's refactor-every-step benchmark mode, Sec. 3): column j of
    a..e (each of shape (n, batch), row-indexed like `Diagonals`, batch
    fastest) is the matrix of system j, column j of F its right-hand side.
    Each system goes through the Sec. 2.4 factorisation and sweeps above.
    Raises SystemZeroPivot(j, i)."""
    arrs = [np.asarray(x, dtype=np.float64) for x in (a, b, c, d, e)]
    F = np.asarray(F, dtype=np.float64)
    n, m = F.shape
    if any(x.shape != (n, m) for x in arrs):
        raise ValueError("diagonals and F must all have shape (n, batch)")
    X = np.empty_like(F)
    for j in range(m):
        dg = Diagonals(*(np.ascontiguousarray(x[:, j]) for x in arrs))
        try:
            fac = factor(dg)
        except ZeroPivot as exc:
            raise SystemZeroPivot(j, exc.row) from None
        col = np.array(F[:, j:j + 1], order="C", copy=True)  # never the caller's F
        solve_inplace(dg, fac, col)
        X[:, j] = col[:, 0]
    return X
