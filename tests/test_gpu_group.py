"""GPU tests of the batching extension: many matrices in one launch (mode
GROUP_FP64, both kernel variants), the one-solve-per-matrix baseline (mode
GROUP_PER_MATRIX), and captured HIP graphs of several time steps, all
against the CPU oracle."""
import numpy as np
import pytest

import oracle
from oracle import workloads
from paper_1807_07382_amd import inputs
from paper_1807_07382_amd import pentbatch as pb
from tests._gpu import colerr, d4_tol, print_case, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_dev()


SMALL = [(0.01, 64, 8), (3.0, 65, 1), (1e4, 1000, 130), (50.0, 4096, 64), (200.0, 129, 200),
         (0.5, 8192, 5), (7.0, 1, 3), (1e2, 300, 0)]


def make(torch, shapes, seed=0):
    mats = [(s, np.random.Generator(np.random.PCG64(seed + k)).uniform(-1, 1, (n, r)))
            for k, (s, n, r) in enumerate(shapes)]
    plans = [pb.Plan.factor_d4(F.shape[0], s) for s, F in mats]
    Ts = [torch.from_numpy(F.copy()).cuda() for _, F in mats]
    return mats, plans, Ts


@pytest.mark.parametrize("mode", [pb.GROUP_FP64, pb.GROUP_PER_MATRIX])
@pytest.mark.parametrize("steps", [1, 3])
def test_group_small_against_oracle(torch, mode, steps):
    print_case(test="group_small", mode=mode, steps=steps)
    mats, plans, Ts = make(torch, SMALL)
    g = pb.Group(plans)
    for _ in range(steps):
        g.solve_(Ts, mode=mode)
    torch.cuda.synchronize()
    refs = workloads.group_run(mats, steps)
    for (sigma, F), T, ref in zip(mats, Ts, refs):
        X = T.cpu().numpy()
        if F.shape[1]:
            assert np.all(colerr(X, ref) <= steps * d4_tol(sigma)), (sigma, F.shape)
    g.close()
    for p in plans:
        p.close()


def test_group_deterministic_and_ld(torch):
    """Same bits on every launch, and blocks with ld > batch."""
    print_case(test="group_ld")
    shapes = [(2.0, 500, 70), (1e3, 2000, 64)]
    mats = [(s, np.random.Generator(np.random.PCG64(k)).uniform(-1, 1, (n, r)))
            for k, (s, n, r) in enumerate(shapes)]
    plans = [pb.Plan.factor_d4(F.shape[0], s) for s, F in mats]
    bufs = [torch.full((F.shape[0], F.shape[1] + 9), 7.0, dtype=torch.float64, device="cuda")
            for _, F in mats]
    for b, (_, F) in zip(bufs, mats):
        b[:, :F.shape[1]] = torch.from_numpy(F).cuda()
    views = [b[:, :F.shape[1]] for b, (_, F) in zip(bufs, mats)]
    g = pb.Group(plans)
    g.solve_(views)
    first = [v.clone() for v in views]
    for v, (_, F) in zip(views, mats):
        v.copy_(torch.from_numpy(F).cuda())
    g.solve_(views)
    torch.cuda.synchronize()
    for a, b in zip(first, views):
        assert torch.equal(a, b)
    for b, (_, F) in zip(bufs, mats):
        assert bool(torch.all(b[:, F.shape[1]:] == 7.0))
    refs = workloads.group_run(mats, 1)
    for (sigma, _), v, ref in zip(mats, views, refs):
        assert np.all(colerr(v.cpu().numpy(), ref) <= d4_tol(sigma))
    g.close()


@pytest.mark.parametrize("mode,variant", [(pb.GROUP_FP64, 0), (pb.GROUP_PER_MATRIX, 0),
                                          (pb.GROUP_FP64, 1)])
def test_graph_replays_match_eager(torch, mode, variant):
    """A captured graph of 3 steps, replayed 3 times with eager work and
    synchronisations in between: every replay equals the eager result."""
    print_case(test="graph", mode=mode, variant=variant)
    shapes = [(0.3, 200, 33), (5e3, 3000, 100), (1.0, 64, 8)]
    mats, plans, Ts = make(torch, shapes, seed=11)
    g = pb.Group(plans)
    g.set_variant(variant)
    init = [T.clone() for T in Ts]
    # eager reference: 3 steps
    for _ in range(3):
        g.solve_(Ts, mode=mode)
    torch.cuda.synchronize()
    eager = [T.clone() for T in Ts]
    s = torch.cuda.Stream()
    for T, I in zip(Ts, init):
        T.copy_(I)
    torch.cuda.synchronize()
    graph = g.capture(Ts, steps=3, mode=mode, stream=s)
    for rep in range(3):
        for T, I in zip(Ts, init):
            T.copy_(I)
        junk = torch.randn(1000, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        graph.launch(stream=s)
        s.synchronize()
        for T, E in zip(Ts, eager):
            assert torch.equal(T, E), f"replay {rep}"
        del junk
    graph.close()
    refs = workloads.group_run(mats, 3)
    for (sigma, _), E, ref in zip(mats, eager, refs):
        assert np.all(colerr(E.cpu().numpy(), ref) <= 3 * d4_tol(sigma))
    g.close()


def test_group_workload_full_shapes(torch):
    """The 48-matrix workload at its full sizes (sigma_k, N_k, R_k of seed 5),
    5 steps in one persistent launch each; 4 sampled systems per matrix
    against the oracle."""
    print_case(test="group_full")
    mats = inputs.group()
    plans = [pb.Plan.factor_d4(F.shape[0], s) for s, F in mats]
    Ts = [torch.from_numpy(F).cuda() for _, F in mats]
    g = pb.Group(plans)
    steps = 5
    for _ in range(steps):
        g.solve_(Ts)
    torch.cuda.synchronize()
    for k, ((sigma, F), T) in enumerate(zip(mats, Ts)):
        r = F.shape[1]
        cols = np.unique(np.array([0, r // 3, (2 * r) // 3, r - 1]))
        ref = workloads.group_run([(sigma, np.ascontiguousarray(F[:, cols]))], steps)[0]
        X = T[:, torch.from_numpy(cols).cuda()].cpu().numpy()
        assert np.all(colerr(X, ref) <= steps * d4_tol(sigma)), (k, sigma, F.shape)
    g.close()


def test_group_argument_errors(torch):
    L = pb.lib()
    with pb.Plan.factor_d4(10, 1.0) as p:
        arr = (pb._P * 1)(p.handle)
        g = L.pent_group_create(arr, 1)
        assert g
        T = torch.zeros((10, 4), dtype=torch.float64, device="cuda")
        ptrs = (pb._P * 1)(T.data_ptr())
        batch = (pb._I64 * 1)(4)
        ld = (pb._I64 * 1)(3)      # ld < batch
        assert L.pent_group_solve(g, ptrs, batch, ld, 0, None, 0, None) == pb.INVALID_VALUE
        ld = (pb._I64 * 1)(4)
        need = L.pent_group_workspace_size(g, batch)
        assert need > 0
        W = torch.zeros(need, dtype=torch.uint8, device="cuda")
        assert L.pent_group_solve(g, ptrs, batch, ld, 5, W.data_ptr(), need, None) == pb.INVALID_VALUE
        assert L.pent_group_solve(g, ptrs, batch, ld, -1, W.data_ptr(), need, None) == pb.INVALID_VALUE
        # the mixed group mode is declared but not supported (reading of the
        # time-stepping state as FP64); refused before anything is enqueued
        assert (L.pent_group_solve(g, ptrs, batch, ld, pb.GROUP_MIXED, W.data_ptr(), need, None)
                == pb.NOT_SUPPORTED)
        assert L.pent_group_solve(g, ptrs, batch, ld, 0, W.data_ptr(), need - 1, None) == pb.SIZE_MISMATCH
        assert L.pent_group_solve(g, ptrs, batch, ld, 0, W.data_ptr(), need, None) == pb.OK
        assert L.pent_group_destroy(g) == pb.OK
    assert not L.pent_group_create(None, 1)
    assert L.pent_group_destroy(None) == pb.OK


def test_autotune_single_matrix(torch, tmp_path, monkeypatch):
    """The tuner times every schedule on scratch memory, keeps the fastest,
    records it in the cache file, and the tuned solve still matches the
    oracle; a second handle of the same shape reads the cached choice."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PENT_TUNE_CACHE", str(cache))
    n, m, sigma = 1500, 700, 20.0
    print_case(test="autotune", n=n, m=m)
    F = np.random.Generator(np.random.PCG64(3)).uniform(-1, 1, (n, m))
    ref = oracle.solve(oracle.assemble_d4(n, sigma), F)
    with pb.Plan.factor_d4(n, sigma) as p:
        kind, seg, ms = p.autotune(m)
        assert kind in (1, 2, 3, 4) and ms > 0
        assert p.schedule_for(m)[0] == kind
        T = torch.from_numpy(F).cuda()
        p.solve_(T)
        torch.cuda.synchronize()
        assert np.all(colerr(T.cpu().numpy(), ref) <= d4_tol(sigma))
    fields = cache.read_text().split()
    # "arch n batch dtype kind seg_rows ms"
    assert fields[0].startswith("gfx") and fields[1:4] == [str(n), str(m), "0"]
    assert int(fields[4]) == kind and int(fields[5]) == seg
    with pb.Plan.factor_d4(n, sigma) as q:
        assert q.autotune(m)[:2] == (kind, seg)


def test_autotune_group_keeps_data(torch):
    print_case(test="group_autotune")
    shapes = [(0.3, 700, 100), (5e3, 2000, 64), (1.0, 64, 8)]
    mats, plans, Ts = make(torch, shapes, seed=21)
    before = [T.clone() for T in Ts]
    g = pb.Group(plans)
    g.solve_(Ts)                     # bind the caller's buffers first
    torch.cuda.synchronize()
    after_one = [T.clone() for T in Ts]
    v, ms = g.autotune(Ts)
    assert v in (0, 1) and ms > 0
    for a, T in zip(after_one, Ts):
        assert torch.equal(a, T)     # tuning ran on scratch blocks
    g.solve_(Ts)
    torch.cuda.synchronize()
    refs = workloads.group_run(mats, 2)
    for (sigma, _), T, ref in zip(mats, Ts, refs):
        assert np.all(colerr(T.cpu().numpy(), ref) <= 2 * d4_tol(sigma))
    del before
    g.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_group_every_variant(torch, variant):
    """Each kernel variant (the persistent kernel, the single pass) against
    the oracle, two steps."""
    print_case(test="group_variant", variant=variant)
    shapes = [(1e2, 333, 65), (2.0, 4097, 64), (1e4, 100, 7), (0.1, 8192, 3)]
    mats, plans, Ts = make(torch, shapes, seed=31 + variant)
    g = pb.Group(plans)
    g.set_variant(variant)
    g.solve_(Ts)
    g.solve_(Ts)
    torch.cuda.synchronize()
    g.check()
    refs = workloads.group_run(mats, 2)
    for (sigma, _), T, ref in zip(mats, Ts, refs):
        assert np.all(colerr(T.cpu().numpy(), ref) <= 2 * d4_tol(sigma))
    g.close()


def test_group_single_pass_full_shapes(torch):
    """Variant 1 (the single pass over all matrices) on the 48-matrix
    workload at its full sizes, 3 steps; sampled systems against the oracle
    and no timed-out wait."""
    print_case(test="group_full_v1")
    mats = inputs.group()
    plans = [pb.Plan.factor_d4(F.shape[0], s) for s, F in mats]
    Ts = [torch.from_numpy(F).cuda() for _, F in mats]
    g = pb.Group(plans)
    g.set_variant(1)
    steps = 3
    for _ in range(steps):
        g.solve_(Ts)
    torch.cuda.synchronize()
    g.check()
    for k, ((sigma, F), T) in enumerate(zip(mats, Ts)):
        r = F.shape[1]
        cols = np.unique(np.array([0, r // 2, r - 1]))
        ref = workloads.group_run([(sigma, np.ascontiguousarray(F[:, cols]))], steps)[0]
        X = T[:, torch.from_numpy(cols).cuda()].cpu().numpy()
        assert np.all(colerr(X, ref) <= steps * d4_tol(sigma)), (k, sigma, F.shape)
    g.close()


@pytest.mark.parametrize("destroy_group", [False, True])
def test_graph_survives_rebind_and_destroy(torch, destroy_group):
    """A graph keeps the device tables of the binding it was captured with:
    after the group is rebound to other buffers (and then destroyed), the
    old graph still solves its own buffers correctly."""
    print_case(test="graph_rebind", destroy=destroy_group)
    shapes = [(0.3, 300, 70), (5e3, 1500, 64)]
    mats, plans, Ts = make(torch, shapes, seed=41)
    init = [T.clone() for T in Ts]
    g = pb.Group(plans)
    s = torch.cuda.Stream()
    graph = g.capture(Ts, steps=2, stream=s)
    # rebind the group to other buffers of other widths, solve there
    others = [torch.from_numpy(np.random.Generator(np.random.PCG64(50 + k)).uniform(
        -1, 1, (F.shape[0], F.shape[1] + 13))).cuda() for k, (_, F) in enumerate(mats)]
    g.solve_(others)
    g.autotune(others)
    if destroy_group:
        g.close()
    torch.cuda.synchronize()
    for T, I in zip(Ts, init):
        T.copy_(I)
    torch.cuda.synchronize()
    graph.launch(stream=s)
    s.synchronize()
    refs = workloads.group_run(mats, 2)
    for (sigma, _), T, ref in zip(mats, Ts, refs):
        assert np.all(colerr(T.cpu().numpy(), ref) <= 2 * d4_tol(sigma))
    graph.close()
    if not destroy_group:
        g.close()
