"""GPU tests of the 2-D Cahn-Hilliard workload (explicit stencil, x sweeps in
system-major layout, y sweeps batch-fastest) against the oracle's drivers."""
import numpy as np
import pytest

import oracle
from oracle import workloads
from paper_1807_07382_amd import inputs
from paper_1807_07382_amd import pentbatch as pb
from tests._gpu import d4_tol, print_case, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_dev()


@pytest.mark.parametrize("ny,ninst,nx", [(37, 3, 45), (1, 1, 1), (2, 5, 300), (64, 2, 64)])
def test_rhs_stencil(torch, ny, ninst, nx):
    print_case(test="ch2d_rhs", ny=ny, ninst=ninst, nx=nx)
    g = np.random.Generator(np.random.PCG64(ny * nx))
    C = g.uniform(-0.5, 0.5, (ny, ninst, nx))
    dt = g.uniform(1e-7, 1e-5, ninst)
    h = 1.0 / max(nx, 2)
    ref = workloads.ch_rhs(C, dt, h)
    Ct = torch.from_numpy(C).cuda()
    R = torch.empty_like(Ct)
    pb.ch2d_rhs(Ct, R, torch.from_numpy(dt).cuda(), h)
    torch.cuda.synchronize()
    scale = np.max(np.abs(C)) + np.max(np.abs(ref - C))
    assert np.max(np.abs(R.cpu().numpy() - ref)) <= 1e-14 * scale


@pytest.mark.parametrize("steps", [1, 4])
def test_step_small_grid(torch, steps):
    n, ninst, sigma = 96, 3, 200.0
    print_case(test="ch2d_small", steps=steps)
    g = np.random.Generator(np.random.PCG64(7))
    C0 = g.uniform(-0.1, 0.1, (n, ninst, n))
    gam = np.array([1e-3, 1e-2, 1e-1])
    ref = workloads.ch_run(C0, gam, sigma, steps)
    h = 1.0 / n
    dt = torch.from_numpy(sigma * h ** 4 / gam).cuda()
    C = torch.from_numpy(C0.copy()).cuda()
    R = torch.empty_like(C)
    with pb.Plan.factor_d4(n, sigma) as p:
        for _ in range(steps):
            pb.ch2d_step(p, p, C, R, dt, h)
        torch.cuda.synchronize()
    err = np.max(np.abs(C.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= 2 * steps * d4_tol(sigma)


def test_full_grid_sampled_instances(torch):
    """1024 x 1024 grid, 32 instances (the full workload), 5 steps on the
    GPU; instances 0 and 31 against the oracle (instances are independent)."""
    w = inputs.cahn2d()
    n, ninst, sigma = w["nx"], w["ninst"], w["sigma"]
    print_case(test="ch2d_full", n=n, ninst=ninst)
    steps = 5
    h = 1.0 / n
    gam = w["gammas"]
    dt = torch.from_numpy(sigma * h ** 4 / gam).cuda()
    C = torch.from_numpy(w["C0"]).cuda()
    R = torch.empty_like(C)
    with pb.Plan.factor_d4(n, sigma) as p:
        for _ in range(steps):
            pb.ch2d_step(p, p, C, R, dt, h)
        torch.cuda.synchronize()
    for k in (0, ninst - 1):
        sub = np.ascontiguousarray(w["C0"][:, k:k + 1, :])
        ref = workloads.ch_run(sub, gam[k:k + 1], sigma, steps)
        got = C[:, k:k + 1, :].cpu().numpy()
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= 2 * steps * d4_tol(sigma), (k, err)


@pytest.mark.parametrize("ny,ninst,nx", [(96, 3, 96), (70, 2, 130), (37, 3, 45), (5, 1, 300),
                                         (64, 2, 1024), (130, 5, 640), (1024, 32, 1024)])
def test_fused_step_matches_separate_passes(torch, ny, ninst, nx):
    """The step forms the x sweeps' right-hand side inside the sweep kernel;
    it must equal the stencil pass followed by the system-major sweeps bit
    for bit (same point formula, same canonical sweep arithmetic), over
    ragged blocks, tiles that straddle two instances, odd row lengths (no
    16-byte path) and the full grid."""
    print_case(test="ch2d_fused", ny=ny, ninst=ninst, nx=nx)
    g = np.random.Generator(np.random.PCG64(ny * 7919 + nx))
    sigma = 200.0
    C0 = g.uniform(-0.1, 0.1, (ny, ninst, nx))
    h = 1.0 / nx
    dt = torch.from_numpy(sigma * h ** 4 / g.uniform(1e-3, 1e-1, ninst)).cuda()
    C = torch.from_numpy(C0).cuda()
    R = torch.empty_like(C)
    R2 = torch.empty_like(C)
    with pb.Plan.factor_d4(nx, sigma) as px, pb.Plan.factor_d4(ny, sigma) as py:
        pb.ch2d_rhs(C, R2, dt, h)
        px.solve_strided_(R2.view(ny * ninst, nx))
        pb.ch2d_step(px, py, C, R, dt, h)
        torch.cuda.synchronize()
        px.check()
    assert torch.equal(R, R2)


@pytest.mark.parametrize("ny,ninst,nx", [(64, 2, 256), (200, 3, 1024)])
def test_fused_step_misaligned_buffers(torch, ny, ninst, nx):
    """C and R one double past a 16-byte boundary: the kernel takes its
    element-by-element path for every block; the result must equal the
    aligned run's bit for bit."""
    print_case(test="ch2d_misaligned", ny=ny, ninst=ninst, nx=nx)
    g = np.random.Generator(np.random.PCG64(nx + 3 * ny))
    sigma = 200.0
    C0 = g.uniform(-0.1, 0.1, (ny, ninst, nx))
    h = 1.0 / nx
    dt = torch.from_numpy(sigma * h ** 4 / g.uniform(1e-3, 1e-1, ninst)).cuda()
    size = ny * ninst * nx
    Ca = torch.from_numpy(C0).cuda()
    Ra = torch.empty_like(Ca)
    bufc = torch.empty(size + 1, dtype=torch.float64, device="cuda")
    bufr = torch.empty(size + 1, dtype=torch.float64, device="cuda")
    Cm = bufc[1:].view(ny, ninst, nx)
    Rm = bufr[1:].view(ny, ninst, nx)
    assert Cm.data_ptr() % 16 == 8 and Cm.is_contiguous()
    Cm.copy_(Ca)
    with pb.Plan.factor_d4(nx, sigma) as px, pb.Plan.factor_d4(ny, sigma) as py:
        pb.ch2d_step(px, py, Ca, Ra, dt, h)
        pb.ch2d_step(px, py, Cm, Rm, dt, h)
        torch.cuda.synchronize()
        px.check()
    assert torch.equal(Rm, Ra)
    assert torch.equal(Cm, Ca)
