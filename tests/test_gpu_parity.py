"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Factorisation and assembly are compared bit for bit;
solves element by element within the tolerance of tests/_gpu.py, plus the
backward-error gate eta <= 1e-12 (compensated residual)."""
import numpy as np
import pytest

import oracle
from oracle import workloads
from paper_1807_07382_amd import inputs
from paper_1807_07382_amd import pentbatch as pb
from tests._gpu import colerr, d4_tol, print_case, torch_dev
from tests.test_oracle_pins import random_dd

pytestmark = pytest.mark.gpu

SCHEDULES = [(1, 0), (2, 16), (2, 32), (2, 64), (3, 0), (4, 32), (4, 64)]


@pytest.fixture(scope="module")
def torch():
    return torch_dev()


def solve_gpu(torch, plan, F, kind=0, seg=0, ld=None):
    """Solve on the GPU with a forced schedule; returns (X, padding after)."""
    n, m = F.shape
    ld = m if ld is None else ld
    buf = np.random.Generator(np.random.PCG64(99)).uniform(-9, 9, (n, ld))
    buf[:, :m] = F
    T = torch.from_numpy(buf).cuda()
    plan.set_schedule(kind, seg)
    plan.solve_(T[:, :m])
    torch.cuda.synchronize()
    out = T.cpu().numpy()
    return out[:, :m], (out[:, m:], buf[:, m:])


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 257, 4096])
@pytest.mark.parametrize("sigma", [0.0, 0.1, 50.0, 200.0, 1e4])
def test_assembly_and_factors_bitwise(torch, n, sigma):
    print_case(test="factor_d4", n=n, sigma=sigma)
    with pb.Plan.factor_d4(n, sigma) as p:
        dg = oracle.assemble_d4(n, sigma)
        for got, ref in zip(p.diagonals(), dg):
            assert np.array_equal(got, ref)
        fac = oracle.factor(dg)
        for got, ref in zip(p.factors(), fac):
            assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,sigma", [(8192, 50.0), (8192, 1e4), (20000, 1e5), (777, 3.0), (130, 7.0)])
def test_long_factors_bitwise(torch, n, sigma):
    """Long constant-coefficient factorisations, where the device copies the
    rows of the recurrence's exact cycle instead of recomputing them: the
    same bits as the oracle's row-by-row recurrence."""
    print_case(test="factor_long", n=n, sigma=sigma)
    with pb.Plan.factor_d4(n, sigma) as p:
        fac = oracle.factor(oracle.assemble_d4(n, sigma))
        for got, ref in zip(p.factors(), fac):
            assert np.array_equal(got, ref)


def test_piecewise_constant_factors_bitwise(torch):
    """Diagonals constant on three stretches (the cycle breaks where a
    stretch ends and the serial recurrence resumes), non-symmetric, plus a
    stretch of random rows: factors bit for bit against the oracle."""
    n = 9000
    print_case(test="factor_piecewise", n=n)
    g = np.random.Generator(np.random.PCG64(31))
    rows = [(0, 3000, (0.5, -2.0, 9.0, -1.5, 0.25)), (3000, 3500, None),
            (3500, 7000, (1.0, -4.0, 10.0, -3.0, 0.75)), (7000, n, (2.0, 1.0, 12.0, 1.0, -2.0))]
    dg = [np.zeros(n) for _ in range(5)]
    for r0, r1, vals in rows:
        for q in range(5):
            if vals is None:
                dg[q][r0:r1] = g.uniform(-1, 1, r1 - r0)
                if q == 2:
                    dg[q][r0:r1] += 6.0
            else:
                dg[q][r0:r1] = vals[q]
    with pb.Plan.factor(*dg) as p:
        fac = oracle.factor(oracle.Diagonals(*dg))
        for got, ref in zip(p.factors(), fac):
            assert np.array_equal(got, ref)


@pytest.mark.parametrize("n", [1, 2, 7, 300])
def test_general_factors_bitwise(torch, n):
    print_case(test="factor_general", n=n)
    dg = random_dd(n, seed=n)
    with pb.Plan.factor(*dg) as p:
        for got, ref in zip(p.factors(), oracle.factor(dg)):
            assert np.array_equal(got, ref)


def test_zero_pivot_rows(torch):
    print_case(test="zero_pivot")
    dg = oracle.assemble_d4(6, 1.0)
    dg.c[0] = 0.0
    with pytest.raises(pb.ZeroPivotError) as ei:
        pb.Plan.factor(*dg)
    assert ei.value.row == 0
    sing = (np.zeros(2), np.array([0.0, 1.0]), np.array([1.0, 1.0]), np.array([1.0, 0.0]),
            np.zeros(2))
    with pytest.raises(pb.ZeroPivotError) as ei:
        pb.Plan.factor(*sing)
    assert ei.value.row == 1
    dg = oracle.assemble_d4(8, 1.0)
    dg.c[5] = np.inf
    with pytest.raises(pb.ZeroPivotError) as ei:
        pb.Plan.factor(*dg)
    assert ei.value.row == 5


@pytest.mark.parametrize("kind,seg", SCHEDULES)
def test_plain_workload(torch, kind, seg):
    """N=256, sigma=0.1, 256 RHS: the whole output against the oracle."""
    w = inputs.plain()
    print_case(test="plain", kind=kind, seg=seg)
    ref = oracle.solve(oracle.assemble_d4(w["n"], w["sigma"]), w["F"])
    with pb.Plan.factor_d4(w["n"], w["sigma"]) as p:
        X, _ = solve_gpu(torch, p, w["F"], kind, seg)
    assert np.all(colerr(X, ref) <= d4_tol(w["sigma"]))
    eta, _ = oracle.residual(oracle.assemble_d4(w["n"], w["sigma"]), X, w["F"])
    assert np.all(eta <= 1e-12)


@pytest.mark.parametrize("kind,seg", SCHEDULES)
@pytest.mark.parametrize("n,m,pad", [(1, 5, 0), (2, 3, 1), (3, 64, 0), (5, 65, 3), (17, 1, 7),
                                     (63, 127, 1), (64, 64, 64), (65, 200, 0), (100, 63, 5),
                                     (257, 129, 0), (1000, 300, 20)])
def test_ragged_sizes(torch, kind, seg, n, m, pad):
    print_case(test="ragged", kind=kind, seg=seg, n=n, m=m, pad=pad)
    sigma = 3.0
    F = np.random.Generator(np.random.PCG64(n * 1000 + m)).uniform(-1, 1, (n, m))
    ref = oracle.solve(oracle.assemble_d4(n, sigma), F)
    with pb.Plan.factor_d4(n, sigma) as p:
        X, (after, before) = solve_gpu(torch, p, F, kind, seg, ld=m + pad)
    assert np.all(colerr(X, ref) <= d4_tol(sigma))
    assert np.array_equal(after, before), "columns past the batch were modified"


@pytest.mark.parametrize("kind,seg", SCHEDULES)
@pytest.mark.parametrize("sigma", [0.1, 50.0, 1e4])
def test_general_nonsymmetric(torch, kind, seg, sigma):
    """Non-symmetric diagonally dominant matrix with random-sign diagonal."""
    n, m = 777, 130
    print_case(test="general", kind=kind, seg=seg, sigma=sigma)
    dg = random_dd(n, seed=int(sigma * 10) + 1)
    F = np.random.Generator(np.random.PCG64(5)).uniform(-1, 1, (n, m))
    ref = oracle.solve(dg, F)
    with pb.Plan.factor(*dg) as p:
        X, _ = solve_gpu(torch, p, F, kind, seg)
    assert np.all(colerr(X, ref) <= 1e-13)
    eta, _ = oracle.residual(dg, X, F)
    assert np.all(eta <= 1e-15)


@pytest.mark.parametrize("kind,seg", SCHEDULES)
def test_column_bits_independent_of_position(torch, kind, seg):
    """A fixed schedule gives the same bits for a system wherever it sits in
    the batch and whatever ld is."""
    n = 300
    print_case(test="position", kind=kind, seg=seg)
    g = np.random.Generator(np.random.PCG64(3))
    col = g.uniform(-1, 1, n)
    outs = []
    with pb.Plan.factor_d4(n, 50.0) as p:
        for m, pos, pad in [(1, 0, 0), (64, 17, 0), (300, 299, 9), (130, 64, 1)]:
            F = g.uniform(-1, 1, (n, m))
            F[:, pos] = col
            X, _ = solve_gpu(torch, p, F, kind, seg, ld=m + pad)
            outs.append(X[:, pos].copy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("n", [1024, 1025, 2048, 2049, 4095, 4096, 4097, 5000])
@pytest.mark.parametrize("m,pad", [(13, 7), (64, 0), (200, 3)])
def test_tile_row_boundaries(torch, n, m, pad):
    """Resident tile at the sizes where rows per lane switch (16/32/64) and
    just past its limit (n > 4096 falls back to the partitioned sweep)."""
    print_case(test="tile_bounds", n=n, m=m, pad=pad)
    sigma = 1e4
    F = np.random.Generator(np.random.PCG64(n + m)).uniform(-1, 1, (n, m))
    ref = oracle.solve(oracle.assemble_d4(n, sigma), F)
    with pb.Plan.factor_d4(n, sigma) as p:
        X, (after, before) = solve_gpu(torch, p, F, 3, 0, ld=m + pad)
    assert np.all(colerr(X, ref) <= d4_tol(sigma))
    assert np.array_equal(after, before)


def test_batch_zero_is_noop(torch):
    with pb.Plan.factor_d4(16, 1.0) as p:
        assert pb.lib().pent_solve(p.handle, None, 0, 0, None) == pb.OK
        T = torch.zeros((16, 0), dtype=torch.float64, device="cuda")
        p.solve_(T)


def test_solve_argument_errors(torch):
    with pb.Plan.factor_d4(16, 1.0) as p:
        T = torch.zeros((16, 8), dtype=torch.float64, device="cuda")
        L = pb.lib()
        assert L.pent_solve(p.handle, T.data_ptr(), 8, 7, None) == pb.INVALID_VALUE
        assert L.pent_solve(p.handle, T.data_ptr(), -1, 8, None) == pb.INVALID_VALUE
        assert L.pent_solve(p.handle, None, 8, 8, None) == pb.INVALID_VALUE
        assert L.pent_solve_strided(p.handle, T.data_ptr(), 1, 15, None) == pb.INVALID_VALUE
        assert L.pent_set_schedule(p.handle, 2, 48) == pb.INVALID_VALUE
        assert L.pent_set_schedule(p.handle, 9, 0) == pb.INVALID_VALUE
        assert L.pent_set_schedule(p.handle, 4, 16) == pb.INVALID_VALUE


@pytest.mark.parametrize("n,m,pad", [(1, 3, 0), (5, 64, 2), (33, 65, 0), (1024, 100, 8),
                                     (1000, 130, 3)])
def test_strided_layout(torch, n, m, pad):
    """System-major storage: system j = n contiguous values at F + j*ld."""
    print_case(test="strided", n=n, m=m, pad=pad)
    sigma = 200.0
    g = np.random.Generator(np.random.PCG64(n + m))
    buf = g.uniform(-1, 1, (m, n + pad))
    ref = oracle.solve(oracle.assemble_d4(n, sigma), np.ascontiguousarray(buf[:, :n].T))
    T = torch.from_numpy(buf.copy()).cuda()
    with pb.Plan.factor_d4(n, sigma) as p:
        p.solve_strided_(T[:, :n])
        torch.cuda.synchronize()
    out = T.cpu().numpy()
    assert np.all(colerr(np.ascontiguousarray(out[:, :n].T), ref) <= d4_tol(sigma))
    assert np.array_equal(out[:, n:], buf[:, n:])


@pytest.mark.parametrize("n,m,pad", [(4133, 1000, 5), (1024, 4100, 0)])
def test_strided_single_pass_deterministic(torch, n, m, pad):
    """System-major solves by the single pass (blocks transposed through
    LDS): the same bits on every run, oracle parity, padding untouched, no
    timed-out wait; a ragged last tile of systems and a ragged last group of
    rows."""
    print_case(test="strided_det", n=n, m=m, pad=pad)
    sigma = 50.0
    buf = np.random.Generator(np.random.PCG64(n * m)).uniform(-1, 1, (m, n + pad))
    ref = oracle.solve(oracle.assemble_d4(n, sigma), np.ascontiguousarray(buf[:, :n].T))
    outs = []
    with pb.Plan.factor_d4(n, sigma) as p:
        for _ in range(3):
            T = torch.from_numpy(buf.copy()).cuda()
            p.solve_strided_(T[:, :n])
            outs.append(T)
        torch.cuda.synchronize()
        p.check()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    out = outs[0].cpu().numpy()
    assert np.all(colerr(np.ascontiguousarray(out[:, :n].T), ref) <= d4_tol(sigma))
    assert np.array_equal(out[:, n:], buf[:, n:])


def test_hyperdiff_full_size_sampled(torch):
    """The hyperdiffusion workload at full size (N=4096, 65536 systems, the
    automatic schedule the benchmark uses), two backward-Euler steps; 256
    sampled systems against the oracle and the contraction property on all."""
    w = inputs.hyperdiff()
    n, sigma = w["n"], w["sigma"]
    print_case(test="hyperdiff_full", n=n, batch=w["C0"].shape[1])
    cols = np.random.Generator(np.random.PCG64(77)).choice(w["C0"].shape[1], 256, replace=False)
    cols = np.concatenate([cols, [0, 63, 64, w["C0"].shape[1] - 1]])
    T = torch.from_numpy(w["C0"]).cuda()
    norm0 = torch.linalg.vector_norm(T, dim=0)
    with pb.Plan.factor_d4(n, sigma) as p:
        p.solve_(T)
        p.solve_(T)
        torch.cuda.synchronize()
    norm2 = torch.linalg.vector_norm(T, dim=0)
    assert bool(torch.all(norm2 <= norm0))
    X = T[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    ref = workloads.hyperdiffusion(n, sigma, w["C0"][:, cols], 2)
    assert np.all(colerr(X, ref) <= 2 * d4_tol(sigma))


@pytest.mark.parametrize("seg", [32, 64])
@pytest.mark.parametrize("n,m", [(4133, 1000), (700, 4097), (64, 130)])
def test_single_pass_deterministic(torch, seg, n, m):
    """The single-pass schedule gives the same bits on every run (the
    look-back replays the serial interface chain whatever the timing), agrees
    with the oracle, and reports no timed-out wait."""
    print_case(test="onepass_det", seg=seg, n=n, m=m)
    F = np.random.Generator(np.random.PCG64(n + m)).uniform(-1, 1, (n, m))
    ref = oracle.solve(oracle.assemble_d4(n, 50.0), F)
    with pb.Plan.factor_d4(n, 50.0) as p:
        p.set_schedule(4, seg)
        assert p.schedule_for(m) == (4, seg)
        outs = []
        for _ in range(3):
            T = torch.from_numpy(F).cuda()
            p.solve_(T)
            outs.append(T)
        torch.cuda.synchronize()
        p.check()
        for o in outs[1:]:
            assert torch.equal(o, outs[0])
        assert np.all(colerr(outs[0].cpu().numpy(), ref) <= d4_tol(50.0))


@pytest.mark.parametrize("seg", [32, 64])
def test_single_pass_full_hyperdiff(torch, seg):
    """The single-pass schedule on the full hyperdiffusion workload (N=4096,
    65536 systems: 1024 tiles), two steps; sampled systems against the
    oracle, the contraction property on all, no timed-out wait."""
    w = inputs.hyperdiff()
    n, sigma = w["n"], w["sigma"]
    print_case(test="onepass_full", seg=seg)
    cols = np.random.Generator(np.random.PCG64(78)).choice(w["C0"].shape[1], 128, replace=False)
    cols = np.concatenate([cols, [0, 63, 64, w["C0"].shape[1] - 1]])
    T = torch.from_numpy(w["C0"]).cuda()
    norm0 = torch.linalg.vector_norm(T, dim=0)
    with pb.Plan.factor_d4(n, sigma) as p:
        p.set_schedule(4, seg)
        assert p.schedule_for(T.shape[1]) == (4, seg)
        p.solve_(T)
        p.solve_(T)
        torch.cuda.synchronize()
        p.check()
    assert bool(torch.all(torch.linalg.vector_norm(T, dim=0) <= norm0))
    X = T[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    ref = workloads.hyperdiffusion(n, sigma, w["C0"][:, cols], 2)
    assert np.all(colerr(X, ref) <= 2 * d4_tol(sigma))


@pytest.mark.parametrize("seg", [32, 64])
@pytest.mark.parametrize("n,m,extra", [(1024, 64, 0), (1500, 1000, 64), (4097, 333, 8)])
def test_tiled_layout_equals_interleaved(torch, seg, n, m, extra):
    """pent_solve_tiled (each 64-system tile its own interleaved block, with
    padding between tiles) gives every system the bits pent_solve gives it in
    the ordinary interleaved layout (same single-pass kernel, same
    arithmetic); the padding is not touched; sampled systems against the
    oracle."""
    import ctypes
    print_case(test="tiled", n=n, m=m, seg=seg)
    rng = np.random.default_rng(7)
    sigma = 50.0
    F = rng.uniform(-1, 1, (n, m))
    tiles = (m + 63) // 64
    ts = n * 64 + extra
    buf = rng.uniform(-9, 9, tiles * ts)
    Fp = np.zeros((n, tiles * 64))
    Fp[:, :m] = F
    for t in range(tiles):
        blk = buf[t * ts: t * ts + n * 64].reshape(n, 64)
        cols = min(64, m - 64 * t)
        blk[:, :cols] = F[:, 64 * t: 64 * t + cols]
    T = torch.from_numpy(buf.copy()).cuda()
    with pb.Plan.factor_d4(n, sigma) as plan:
        plan.set_schedule(4, seg)
        st = pb.lib().pent_solve_tiled(plan.handle, ctypes.c_void_p(T.data_ptr()), m, 64, ts,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == pb.OK
        R = torch.from_numpy(F.copy()).cuda()
        plan.solve_(R)
        torch.cuda.synchronize()
        plan.check()
    out = T.cpu().numpy()
    ref = R.cpu().numpy()
    for t in range(tiles):
        cols = min(64, m - 64 * t)
        blk = out[t * ts: t * ts + n * 64].reshape(n, 64)
        assert np.array_equal(blk[:, :cols], ref[:, 64 * t: 64 * t + cols]), f"tile {t}"
        orig = buf[t * ts: t * ts + n * 64].reshape(n, 64)
        assert np.array_equal(blk[:, cols:], orig[:, cols:])  # idle columns of a partial tile
        assert np.array_equal(out[t * ts + n * 64:(t + 1) * ts], buf[t * ts + n * 64:(t + 1) * ts])
    cols = np.unique(np.linspace(0, m - 1, 12).astype(np.int64))
    oref = oracle.solve(oracle.assemble_d4(n, sigma), F[:, cols])
    assert np.max(colerr(ref[:, cols], oref)) <= d4_tol(sigma)


def test_tiled_layout_argument_errors(torch):
    import ctypes
    with pb.Plan.factor_d4(2048, 1.0) as plan:
        T = torch.zeros(2048 * 64, dtype=torch.float64, device="cuda")
        p = ctypes.c_void_p(T.data_ptr())
        L = pb.lib()
        assert L.pent_solve_tiled(plan.handle, p, 64, 63, 2048 * 64, None) == pb.INVALID_VALUE
        assert L.pent_solve_tiled(plan.handle, p, 64, 64, 2047 * 64 + 63, None) == pb.INVALID_VALUE
        assert L.pent_solve_tiled(plan.handle, p, -1, 64, 2048 * 64, None) == pb.INVALID_VALUE
        assert L.pent_solve_tiled(plan.handle, None, 64, 64, 2048 * 64, None) == pb.INVALID_VALUE
        assert L.pent_solve_tiled(plan.handle, None, 0, 64, 2048 * 64, None) == pb.OK
        plan.set_schedule(2, 64)  # not the single pass
        assert L.pent_solve_tiled(plan.handle, p, 64, 64, 2048 * 64, None) == pb.NOT_SUPPORTED
        torch.cuda.synchronize()
        assert torch.count_nonzero(T).item() == 0
