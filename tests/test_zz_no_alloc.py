"""pent_solve_noalloc (the solve whose scratch is the library's fixed device
buffer instead of an allocation) against pent_solve, called through the C
ABI: the same schedule and kernels, so the results must agree bit for bit;
a sample of systems is also checked against the oracle.  Consecutive calls
share the buffer, so each following call is smaller than the one before (it
must not see the earlier call's status words or carries)."""
import ctypes

import numpy as np
import pytest

from paper_1807_07382_amd import inputs
from paper_1807_07382_amd import pentbatch as pb
from tests._gpu import colerr, d4_tol, print_case, torch_dev

pytestmark = pytest.mark.gpu


def _noalloc(plan, buf, batch):
    """pent_solve_noalloc on the first `batch` columns of buf (ld = its row
    stride) on torch's current stream."""
    torch = torch_dev()
    return pb.lib().pent_solve_noalloc(plan.handle, ctypes.c_void_p(buf.data_ptr()), int(batch),
                                       buf.stride(0),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _pair(plan, F0, batch, orc, sigma, sample):
    """noalloc and pent_solve on copies of F0 (columns past `batch` are
    padding of the leading dimension and must stay untouched): equal bits,
    sampled columns against the oracle."""
    torch = torch_dev()
    A = F0.clone()
    B = F0.clone()
    assert _noalloc(plan, A, batch) == pb.OK
    plan.solve_(B[:, :batch])
    torch.cuda.synchronize()
    pb._check(pb.lib().pent_check(plan.handle), "check")
    assert torch.equal(A, B), "noalloc result differs from pent_solve"
    assert torch.equal(A[:, batch:], F0[:, batch:])
    cols = np.unique(np.linspace(0, batch - 1, sample).astype(np.int64))
    f = F0[:, cols].cpu().numpy()
    ref = orc.solve(orc.assemble_d4(plan.n, sigma), f)
    assert np.max(colerr(A[:, cols].cpu().numpy(), ref)) <= d4_tol(sigma)


def test_noalloc_equals_solve_two_calls_shrinking(orc):
    torch = torch_dev()
    rng = np.random.default_rng(11)
    n, sigma = 4096, 50.0
    with pb.Plan.factor_d4(n, sigma) as plan:
        kind, seg = ctypes.c_int(), ctypes.c_int()
        pb.lib().pent_query_schedule(plan.handle, 65536, ctypes.byref(kind), ctypes.byref(seg))
        assert (kind.value, seg.value) == (4, 64)  # the single pass: scratch in use
        print_case(test="noalloc", n=n, batch=65536, call=1)
        F0 = torch.empty((n, 65536), dtype=torch.float64, device="cuda").uniform_(-1, 1)
        _pair(plan, F0, 65536, orc, sigma, 6)
        del F0
        # second call: smaller and ragged (batch not a multiple of 64, ld > batch)
        print_case(test="noalloc", n=n, batch=1000, ld=1024, call=2)
        G = torch.from_numpy(rng.uniform(-1, 1, (n, 1024))).to("cuda")
        _pair(plan, G, 1000, orc, sigma, 1000)


def test_noalloc_other_schedules_and_limits(orc):
    torch = torch_dev()
    rng = np.random.default_rng(12)
    # small solve: the resident tile (no scratch at all)
    print_case(test="noalloc", n=256, batch=256, schedule="auto")
    w = inputs.plain()
    with pb.Plan.factor_d4(w["n"], w["sigma"]) as plan:
        _pair(plan, torch.from_numpy(w["F"]).to("cuda"), 256, orc, w["sigma"], 256)
    n, sigma = 2048, 200.0
    with pb.Plan.factor_d4(n, sigma) as plan:
        # partitioned, 64-row segments (tables built by pent_factor)
        plan.set_schedule(2, 64)
        print_case(test="noalloc", n=n, batch=3000, schedule="2,64")
        _pair(plan, torch.from_numpy(rng.uniform(-1, 1, (n, 3000))).to("cuda"), 3000, orc, sigma,
              300)
        # a schedule whose tables do not exist yet is refused (no lazy build)
        plan.set_schedule(2, 16)
        F = torch.from_numpy(rng.uniform(-1, 1, (n, 200))).to("cuda")
        before = F.clone()
        assert _noalloc(plan, F, 200) == pb.NOT_SUPPORTED
        torch.cuda.synchronize()
        assert torch.equal(F, before)
        plan.solve_(F.clone())  # builds them
        torch.cuda.synchronize()
        print_case(test="noalloc", n=n, batch=200, schedule="2,16")
        _pair(plan, before, 200, orc, sigma, 200)
    # more single-pass units than the buffer holds: refused before any launch
    with pb.Plan.factor_d4(4096, 50.0) as plan:
        F = torch.zeros((4096, 8), dtype=torch.float64, device="cuda")
        st = pb.lib().pent_solve_noalloc(plan.handle, ctypes.c_void_p(F.data_ptr()), 80000, 80000,
                                         None)
        assert st == pb.NOT_SUPPORTED
        torch.cuda.synchronize()
        assert torch.count_nonzero(F).item() == 0
