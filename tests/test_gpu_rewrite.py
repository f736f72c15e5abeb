"""GPU tests of the per-system refactor-and-solve (pent_solve_rewrite)
against the CPU oracle's rewrite_solve on the same seeded inputs."""
import numpy as np
import pytest

import oracle
from paper_1807_07382_amd import pentbatch as pb
from tests._gpu import U, colerr, d4_tol, print_case, torch_dev
from tests.test_oracle_rewrite import per_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_dev()


def varah_kappa_cols(diags):
    a, b, c, d, e = diags
    off = np.abs(a) + np.abs(b) + np.abs(d) + np.abs(e)
    return np.max(off + np.abs(c), axis=0) / np.min(np.abs(c) - off, axis=0)


def to_dev(torch, x, ld):
    """(n, m) array into a device buffer with row stride ld >= m (padding 7)."""
    n, m = x.shape
    buf = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda")
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return buf


@pytest.mark.parametrize("n,m,pad", [(1, 3, 0), (2, 1, 2), (3, 64, 0), (5, 65, 1), (8, 9, 0),
                                     (9, 130, 3), (17, 300, 0), (100, 64, 5), (1000, 257, 0),
                                     (4099, 70, 2)])
def test_rewrite_against_oracle(torch, n, m, pad):
    print_case(test="rewrite", n=n, m=m, pad=pad)
    diags = per_system(n, m, seed=n * 7 + m)
    F = np.random.Generator(np.random.PCG64(n + m)).uniform(-1, 1, (n, m))
    ref = oracle.rewrite_solve(*diags, F)
    dev = [to_dev(torch, x, m + pad) for x in diags]
    Fd = to_dev(torch, F, m + 2 * pad)
    views = [x[:, :m] for x in dev]
    pb.solve_rewrite_(*views, Fd[:, :m], check=True)
    torch.cuda.synchronize()
    X = Fd[:, :m].cpu().numpy()
    assert np.all(colerr(X, ref) <= 64 * U * varah_kappa_cols(diags))
    assert bool(torch.all(Fd[:, m:] == 7.0))
    for x, h in zip(dev, diags):   # the diagonals are only read
        assert np.array_equal(x[:, :m].cpu().numpy(), h)


@pytest.mark.parametrize("n", [64, 1024])
def test_rewrite_per_system_sigma(torch, n):
    """Systems I + sigma_j D4 with sigma_j log-uniform in [1e-2, 1e4]."""
    m = 200
    print_case(test="rewrite_sigma", n=n)
    sig = 10.0 ** np.random.Generator(np.random.PCG64(n)).uniform(-2, 4, m)
    cols = [oracle.assemble_d4(n, s) for s in sig]
    diags = [np.stack([getattr(dg, k) for dg in cols], axis=1) for k in "abcde"]
    F = np.random.Generator(np.random.PCG64(n + 1)).uniform(-1, 1, (n, m))
    ref = oracle.rewrite_solve(*diags, F)
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in diags]
    Fd = torch.from_numpy(F.copy()).cuda()
    pb.solve_rewrite_(*dev, Fd, check=True)
    torch.cuda.synchronize()
    err = colerr(Fd.cpu().numpy(), ref)
    assert np.all(err <= np.array([d4_tol(s) for s in sig]))


def test_rewrite_zero_pivot_reported(torch):
    """System 1 meets alpha_1 = 0 exactly, system 3 alpha_0 = 0: the check
    names system 1, row 1; the other systems are still solved."""
    n, m = 10, 5
    a, b, c, d, e = (x.copy() for x in per_system(n, m, seed=9))
    c[0, 1], d[0, 1], b[1, 1], c[1, 1] = 1.0, 2.0, 3.0, 6.0
    c[0, 3] = 0.0
    print_case(test="rewrite_pivot")
    F = np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, (n, m))
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (a, b, c, d, e)]
    Fd = torch.from_numpy(F.copy()).cuda()
    with pytest.raises(pb.SystemZeroPivotError) as ei:
        pb.solve_rewrite_(*dev, Fd, check=True)
    assert (ei.value.system, ei.value.row) == (1, 1)
    good = [0, 2, 4]
    ref = oracle.rewrite_solve(*(x[:, good] for x in (a, b, c, d, e)), F[:, good])
    X = Fd.cpu().numpy()[:, good]
    assert np.all(colerr(X, ref) <= 1e-13)


def test_rewrite_shared_matrix_matches_constant_path(torch):
    """All systems with the same matrix: the rewrite path and the
    factor-once path agree within the parity tolerance."""
    n, m, sigma = 2000, 130, 50.0
    print_case(test="rewrite_shared")
    dg = oracle.assemble_d4(n, sigma)
    diags = [np.repeat(getattr(dg, k)[:, None], m, axis=1) for k in "abcde"]
    F = np.random.Generator(np.random.PCG64(2)).uniform(-1, 1, (n, m))
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in diags]
    Fd = torch.from_numpy(F.copy()).cuda()
    pb.solve_rewrite_(*dev, Fd, check=True)
    G = torch.from_numpy(F.copy()).cuda()
    with pb.Plan.factor_d4(n, sigma) as p:
        p.solve_(G)
    torch.cuda.synchronize()
    ref = oracle.solve(dg, F)
    assert np.all(colerr(Fd.cpu().numpy(), ref) <= d4_tol(sigma))
    assert np.all(colerr(Fd.cpu().numpy(), G.cpu().numpy()) <= 2 * d4_tol(sigma))


def test_rewrite_workload_full_size_sampled(torch):
    """The per-system-matrix workload at full size (N = 1024, 65536 systems,
    system j = I + sigma_j D4 with sigma_j log-uniform in [1e-2, 1e4]; the
    inputs and the workspace call that the benchmark times), two steps, the
    second refactoring and solving again from the first one's output.
    Sampled systems (both ends of the batch and of 64-system tiles) against
    the oracle, whose second step starts from its own first step."""
    from paper_1807_07382_amd import inputs
    w = inputs.rewrite()
    n, batch = w["n"], w["sigma"].shape[0]
    print_case(test="rewrite_full", n=n, batch=batch)
    sig = torch.from_numpy(w["sigma"]).cuda()
    ones = torch.ones((n, 1), dtype=torch.float64, device="cuda")
    diags = [ones * sig, ones * (-4.0 * sig), 1.0 + 6.0 * ones * sig, ones * (-4.0 * sig),
             ones * sig]
    F = torch.from_numpy(w["F"]).cuda()
    work = torch.empty(pb.lib().pent_rewrite_workspace_size(n, batch), dtype=torch.uint8,
                       device="cuda")
    cols = np.array([0, 1, 63, 64, 4097, 32768, batch - 65, batch - 2, batch - 1])
    idx = torch.from_numpy(cols).cuda()
    hd = [x[:, idx].cpu().numpy() for x in diags]
    tol = np.array([d4_tol(s) for s in w["sigma"][cols]])
    ref = np.ascontiguousarray(w["F"][:, cols])
    for step in range(2):
        pb.solve_rewrite_(*diags, F, work=work, check=True)
        torch.cuda.synchronize()
        ref = oracle.rewrite_solve(*hd, ref)
        err = colerr(F[:, idx].cpu().numpy(), ref)
        # A^{-1} has norm <= 1 here (SPD, eigenvalues >= 1), so the first
        # step's difference is carried into the second without growth
        assert np.all(err <= (step + 1) * tol), (step, err / tol)
