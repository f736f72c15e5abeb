"""GPU tests of the solves' stream-ordered scratch (the library's own memory
pool, which keeps its memory across synchronisations): many calls of
changing sizes with a synchronisation after each, so freed blocks are
handed out again at other sizes, and two handles solving on two streams at
once, each checked against the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
from oracle import cyclic
from paper_1807_07382_amd import pentbatch as pb
from tests._gpu import colerr, d4_tol, print_case, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_dev()


def rhs(n, m, seed):
    return np.random.Generator(np.random.PCG64(seed)).uniform(-1, 1, (n, m))


def test_scratch_reused_across_sizes(torch):
    """Single-pass solves (scratch grows with the batch) and periodic steps
    of alternating sizes, synchronised after every call."""
    n, sigma = 1500, 20.0
    sizes = [4096, 64, 20000, 1, 777, 20000, 64, 4096]
    dg = oracle.assemble_d4(n, sigma)
    with pb.Plan.factor_d4(n, sigma) as p, pb.Cyclic.factor_d4(n, sigma) as cy:
        p.set_schedule(4, 64)
        cy.set_schedule(2, 64)
        for i, m in enumerate(sizes):
            print_case(test="pool_sizes", call=i, batch=m)
            F = rhs(n, m, seed=100 + i)
            T = torch.from_numpy(F.copy()).cuda()
            p.solve_(T)
            torch.cuda.synchronize()
            p.check()
            cols = np.unique(np.array([0, m // 2, m - 1]))
            ref = oracle.solve(dg, np.ascontiguousarray(F[:, cols]))
            assert np.all(colerr(T.cpu().numpy()[:, cols], ref) <= d4_tol(sigma))
            C = torch.from_numpy(F).cuda()
            X = torch.empty_like(C)
            cy.cn_step(C, X)
            torch.cuda.synchronize()
            cy.check()
            ref = cyclic.cn_run(sigma, np.ascontiguousarray(F[:, cols]), 1)
            got = X.cpu().numpy()[:, cols]
            assert np.max(np.abs(got - ref)) <= 4 * d4_tol(sigma) * np.max(np.abs(F[:, cols]))


def test_two_streams_at_once(torch):
    """Two handles with different matrices solve on two streams without a
    synchronisation between the calls; both results match the oracle."""
    n1, n2, m = 2048, 700, 9000
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    F1, F2 = rhs(n1, m, seed=7), rhs(n2, m, seed=8)
    with pb.Plan.factor_d4(n1, 50.0) as p1, pb.Plan.factor_d4(n2, 0.5) as p2:
        p1.set_schedule(4, 64)
        p2.set_schedule(4, 32)
        T1 = torch.from_numpy(F1.copy()).cuda()
        T2 = torch.from_numpy(F2.copy()).cuda()
        torch.cuda.synchronize()
        for rep in range(3):
            print_case(test="pool_streams", rep=rep)
            T1.copy_(torch.from_numpy(F1))
            T2.copy_(torch.from_numpy(F2))
            torch.cuda.synchronize()
            p1.solve_(T1, stream=s1)
            p2.solve_(T2, stream=s2)
            torch.cuda.synchronize()
            p1.check()
            p2.check()
        cols = np.array([0, 1, 4321, m - 1])
        r1 = oracle.solve(oracle.assemble_d4(n1, 50.0), np.ascontiguousarray(F1[:, cols]))
        r2 = oracle.solve(oracle.assemble_d4(n2, 0.5), np.ascontiguousarray(F2[:, cols]))
        assert np.all(colerr(T1.cpu().numpy()[:, cols], r1) <= d4_tol(50.0))
        assert np.all(colerr(T2.cpu().numpy()[:, cols], r2) <= d4_tol(0.5))
