"""Pins for the oracle's workload drivers (time stepping around the solve)."""
import numpy as np

import oracle
from oracle import workloads

U = np.finfo(np.float64).eps / 2


def test_hyperdiffusion_contracts_every_step():
    """A = I + sigma D4 is SPD with eigenvalues >= 1, so ||A^{-1}||_2 <= 1 and
    every backward-Euler step can only shrink each column's 2-norm."""
    n, m = 512, 16
    C0 = np.random.Generator(np.random.PCG64(2)).uniform(-1, 1, (n, m))
    _, hist = workloads.hyperdiffusion(n, 50.0, C0, 10, norms=True)
    assert np.all(hist[1:] <= hist[:-1] * (1 + 4 * U))
    assert np.all(hist[-1] < hist[0])


def test_hyperdiffusion_matches_dense_steps():
    n, m, sigma = 24, 3, 5.0
    C0 = np.random.Generator(np.random.PCG64(3)).uniform(-1, 1, (n, m))
    A = oracle.dense(oracle.assemble_d4(n, sigma))
    ref = C0.copy()
    for _ in range(4):
        ref = np.linalg.solve(A, ref)
    got = workloads.hyperdiffusion(n, sigma, C0, 4)
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_ch_rhs_matches_loops():
    """5-point Laplacian with zero ghost values, written as plain loops."""
    ny, ninst, nx = 5, 2, 6
    g = np.random.Generator(np.random.PCG64(4))
    C = g.uniform(-0.5, 0.5, (ny, ninst, nx))
    dt = np.array([0.01, 0.03])
    h = 0.25
    got = workloads.ch_rhs(C, dt, h)
    for y in range(ny):
        for k in range(ninst):
            for x in range(nx):
                def w(yy, xx):
                    if 0 <= yy < ny and 0 <= xx < nx:
                        v = C[yy, k, xx]
                        return v ** 3 - v
                    return 0.0
                lap = (w(y, x + 1) + w(y, x - 1) + w(y + 1, x) + w(y - 1, x) - 4 * w(y, x)) / h ** 2
                assert abs(got[y, k, x] - (C[y, k, x] + dt[k] * lap)) <= 1e-15


def test_ch_step_matches_dense_kronecker():
    """x sweep then y sweep == (A_y (x) I)^{-1} (I (x) A_x)^{-1} RHS per instance."""
    n, ninst, sigma = 7, 3, 20.0
    g = np.random.Generator(np.random.PCG64(5))
    C = g.uniform(-0.1, 0.1, (n, ninst, n))
    dt = np.array([1e-3, 2e-3, 5e-4])
    h = 1.0 / n
    dg = oracle.assemble_d4(n, sigma)
    fac = oracle.factor(dg)
    got = workloads.ch_step(C, dt, h, dg, fac)
    A = oracle.dense(dg)
    I = np.eye(n)
    R = workloads.ch_rhs(C, dt, h)
    for k in range(ninst):
        v = R[:, k, :].reshape(-1)                     # y slow, x fast
        v = np.linalg.solve(np.kron(I, A), v)
        v = np.linalg.solve(np.kron(A, I), v)
        assert np.max(np.abs(got[:, k, :].reshape(-1) - v)) <= 1e-14


def test_ch_rhs_constant_field_interior():
    """C^3 - C is constant for a constant field, so the interior Laplacian
    vanishes and only boundary cells (zero ghosts) move."""
    C = np.full((6, 1, 6), 0.3)
    R = workloads.ch_rhs(C, np.array([1e-2]), 0.5)
    assert np.all(R[1:-1, :, 1:-1] == 0.3)
    assert np.all(R[0, :, 1:-1] != 0.3)


def test_group_run_matches_dense():
    mats = [(0.5, np.random.Generator(np.random.PCG64(k)).uniform(-1, 1, (n, r)))
            for k, (n, r) in enumerate([(9, 2), (13, 5), (4, 1)])]
    out = workloads.group_run(mats, 3)
    for (sigma, F), X in zip(mats, out):
        A = oracle.dense(oracle.assemble_d4(F.shape[0], sigma))
        ref = F.copy()
        for _ in range(3):
            ref = np.linalg.solve(A, ref)
        assert np.max(np.abs(X - ref)) <= 1e-14


def test_plain_golden_regression():
    """The oracle still reproduces its committed sample bit for bit."""
    import os
    from paper_1807_07382_amd import inputs
    path = os.path.join(os.path.dirname(__file__), "golden", "plain_oracle_sample.txt")
    w = inputs.plain()
    X = oracle.solve(oracle.assemble_d4(w["n"], w["sigma"]), w["F"])
    for line in open(path):
        if line.startswith("#"):
            continue
        i, j, v = line.split()
        assert X[int(i), int(j)] == float.fromhex(v)
