"""Pins for the oracle's cyclic (periodic) solve and the Crank-Nicolson
hyperdiffusion validation of Sec. 2.3 and Sec. 2.5."""
import os

import numpy as np
import pytest

from oracle import Diagonals, cyclic

U = np.finfo(np.float64).eps / 2


def random_cyclic_dd(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    a, b, d, e = (g.uniform(-1, 1, n) for _ in range(4))
    c = (1.5 * (np.abs(a) + np.abs(b) + np.abs(d) + np.abs(e)) + g.uniform(0.5, 1, n)) \
        * g.choice([-1.0, 1.0], n)
    return Diagonals(a, b, c, d, e)


@pytest.mark.parametrize("n", [5, 6, 7, 8, 13, 40])
def test_cyclic_vs_dense_nonsymmetric(n):
    dg = random_cyclic_dd(n, n)
    F = np.random.Generator(np.random.PCG64(n + 1)).uniform(-1, 1, (n, 4))
    X = cyclic.solve_cyclic(cyclic.bordering(dg), F)
    ref = np.linalg.solve(cyclic.dense_cyclic(dg), F)
    kappa = np.linalg.cond(cyclic.dense_cyclic(dg), 1)
    assert np.max(np.abs(X - ref)) <= 64 * U * kappa * np.max(np.abs(ref))


def test_dense_cyclic_matches_paper_matrix():
    """The first and last two rows of the Sec. 2.3 matrix: (c d e 0 .. 0 a b),
    (b c d e 0 .. 0 a), ..., (e 0 .. 0 a b c d), (d e 0 .. 0 a b c)."""
    n, s = 8, 0.75
    A = cyclic.dense_cyclic(cyclic.cyclic_d4(n, s))
    a, b, c, d, e = s, -4 * s, 1 + 6 * s, -4 * s, s
    z = [0.0] * (n - 5)
    assert list(A[0]) == [c, d, e] + z + [a, b]
    assert list(A[1]) == [b, c, d, e] + z + [a]
    assert list(A[n - 2]) == [e] + z + [a, b, c, d]
    assert list(A[n - 1]) == [d, e] + z + [a, b, c]


@pytest.mark.parametrize("n,sigma,mode", [(16, 3.0, 1), (64, 50.0, 5), (100, 0.1, 7)])
def test_fourier_modes_closed_form(n, sigma, mode):
    """The periodic matrix is circulant: cos(theta j), theta = 2 pi mode / n,
    is an eigenvector with eigenvalue 1 + sigma (2 - 2 cos theta)^2."""
    th = 2 * np.pi * mode / n
    j = np.arange(n)
    f = np.cos(th * j)
    lam = 1 + sigma * (2 - 2 * np.cos(th)) ** 2
    x = cyclic.solve_cyclic(cyclic.bordering(cyclic.cyclic_d4(n, sigma)), f)
    assert np.max(np.abs(x - f / lam)) <= 64 * U * (1 + 16 * sigma)


def test_cn_rhs_is_two_minus_a():
    """f = (2I - A) C, the explicit half of Crank-Nicolson."""
    n, s = 12, 2.5
    C = np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, (n, 3))
    A = cyclic.dense_cyclic(cyclic.cyclic_d4(n, s))
    assert np.max(np.abs(cyclic.cn_rhs(C, s) - (2 * C - A @ C))) <= 1e-13


@pytest.mark.parametrize("n", [16, 64])
def test_cn_steps_closed_form(n):
    """A Fourier mode stays a Fourier mode: after m CN steps it is multiplied
    by G^m, G = (1 - s mu^2) / (1 + s mu^2), mu = 2 - 2 cos(k dx)."""
    dt, T, mode = 1e-8, 1e-5, 2
    C, _, _ = cyclic.hyperdiffusion_cn(n, dt, T, mode)
    dx = 1.0 / n
    s = dt / (2 * dx ** 4)
    mu = 2 - 2 * np.cos(2 * np.pi * mode * dx)
    G = (1 - s * mu * mu) / (1 + s * mu * mu)
    x = dx * np.arange(1, n + 1)
    expect = G ** round(T / dt) * np.cos(2 * np.pi * mode * x)
    assert np.max(np.abs(C - expect)) <= 1e-12


def test_convergence_slope_matches_paper():
    """eps_N(T) at N = 16..256 decays like N^-2; the fitted slope agrees with
    the paper's -2.0162 (golden/convergence.txt) to 0.02."""
    path = os.path.join(os.path.dirname(__file__), "golden", "convergence.txt")
    g = dict(l.split() for l in open(path) if l.strip() and not l.startswith("#"))
    T, dt, mode, slope_paper = float(g["T"]), float(g["dt"]), int(g["mode"]), float(g["slope"])
    Ns = [16, 32, 64, 128, 256]
    eps = [cyclic.hyperdiffusion_cn(n, dt, T, mode)[2] for n in Ns]
    slope = np.polyfit(np.log(Ns), np.log(eps), 1)[0]
    assert abs(slope - float(g["theory"])) < 0.05
    assert abs(slope - slope_paper) < 0.02
