"""Workload oracles (TEST INFRASTRUCTURE ONLY): plain numpy time-stepping
drivers around the oracle's FP64 solve.

* hyperdiffusion: dC/dt = -d^4C/dx^4 (Sec. 2.2, the hyperdiffusion equation
  with gamma = D = L = 1), non-periodic, backward Euler in time, so every step
  solves (I + sigma D4) C^{n+1} = C^n with the factors of one matrix.
* Cahn-Hilliard, 2-D, split implicit: the semi-implicit step of Sec. 2.1
  (explicit D*Lap(C^3 - C), implicit -gamma*D*d^4C) applied direction by
  direction: RHS = C^n + dt*Lap_h(C^3 - C)^n, then (I + sigma D4_x) C* = RHS
  along x, then (I + sigma D4_y) C^{n+1} = C* along y.  Lap_h is the 5-point
  Laplacian with zero ghost values, matching the truncated D4 rows.
* group: many independent matrices, each with its own columns, stepped by
  backward Euler.
"""
from __future__ import annotations

import numpy as np

from . import Diagonals, Factors, assemble_d4, factor, solve_inplace


def hyperdiffusion(n: int, sigma: float, C0: np.ndarray, steps: int,
                   norms: bool = False):
    """Backward-Euler hyperdiffusion: C^{k+1} = (I + sigma D4)^{-1} C^k.
    C0 has shape (n, systems).  Returns the final state (and the per-step
    column 2-norms when ``norms``)."""
    dg = assemble_d4(n, sigma)
    fac = factor(dg)
    C = np.array(C0, dtype=np.float64, order="C", copy=True)
    hist = [np.linalg.norm(C, axis=0)] if norms else None
    for _ in range(steps):
        solve_inplace(dg, fac, C)
        if norms:
            hist.append(np.linalg.norm(C, axis=0))
    return (C, np.array(hist)) if norms else C


def ch_rhs(C: np.ndarray, dt: np.ndarray, h: float) -> np.ndarray:
    """Explicit part of the split Cahn-Hilliard step for a state of shape
    (ny, ninst, nx): RHS = C + dt[k] * Lap_h(C^3 - C), Lap_h the 5-point
    Laplacian over (y, x) with zero ghost values, dt one value per instance."""
    C = np.asarray(C, dtype=np.float64)
    w = C * C * C - C
    p = np.zeros((C.shape[0] + 2, C.shape[1], C.shape[2] + 2))
    p[1:-1, :, 1:-1] = w
    lap = (p[1:-1, :, 2:] + p[1:-1, :, :-2] + p[2:, :, 1:-1] + p[:-2, :, 1:-1]
           - 4.0 * w) / (h * h)
    return C + np.asarray(dt, dtype=np.float64)[None, :, None] * lap


def ch_step(C: np.ndarray, dt: np.ndarray, h: float, dg: Diagonals, fac: Factors) -> np.ndarray:
    """One split-implicit step of the 2-D Cahn-Hilliard workload.  Both
    directions use the same matrix (square grid, one sigma)."""
    ny, ninst, nx = C.shape
    R = ch_rhs(C, dt, h)
    # x direction: unknowns along x, systems (y, inst) -> batch-fastest (nx, ny*ninst)
    Xs = np.ascontiguousarray(R.reshape(ny * ninst, nx).T)
    solve_inplace(dg, fac, Xs)
    Cstar = Xs.T.reshape(ny, ninst, nx)
    # y direction: unknowns along y, systems (inst, x) -> native layout (ny, ninst*nx)
    Ys = np.ascontiguousarray(Cstar.reshape(ny, ninst * nx))
    solve_inplace(dg, fac, Ys)
    return Ys.reshape(ny, ninst, nx)


def ch_run(C0: np.ndarray, gammas: np.ndarray, sigma: float, steps: int) -> np.ndarray:
    """Run the 2-D split Cahn-Hilliard workload on a square grid of spacing
    h = 1/nx (unit domain): sigma = gamma*dt/h^4 is shared by all instances,
    so instance k uses dt_k = sigma*h^4/gamma_k."""
    ny, ninst, nx = C0.shape
    if ny != nx:
        raise ValueError("square grid expected")
    h = 1.0 / nx
    dt = sigma * h ** 4 / np.asarray(gammas, dtype=np.float64)
    dg = assemble_d4(nx, sigma)
    fac = factor(dg)
    C = np.array(C0, dtype=np.float64, copy=True)
    for _ in range(steps):
        C = ch_step(C, dt, h, dg, fac)
    return C


def group_run(mats, steps: int):
    """mats: list of (sigma_k, F_k) with F_k of shape (n_k, r_k).  Every step
    replaces F_k by (I + sigma_k D4)^{-1} F_k.  Returns the final list."""
    out = []
    for sigma, F in mats:
        n = F.shape[0]
        dg = assemble_d4(n, sigma)
        fac = factor(dg)
        X = np.array(F, dtype=np.float64, order="C", copy=True)
        for _ in range(steps):
            solve_inplace(dg, fac, X)
        out.append(X)
    return out
