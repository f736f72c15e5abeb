"""GPU tests of the measurement copies (pent_stream_copy and its other
workgroup shapes): every shape copies an (n x batch) block exactly, leaves
the columns past the batch alone, and is a no-op in place, for sizes that
leave partial tiles, partial row groups and partial workgroups."""
import numpy as np
import pytest

from paper_1807_07382_amd import pentbatch as pb
from tests._gpu import print_case, torch_dev

pytestmark = pytest.mark.gpu

SHAPES = [(1, 4), (1, 2), (2, 2), (2, 1), (4, 1)]


@pytest.fixture(scope="module")
def torch():
    return torch_dev()


@pytest.mark.parametrize("ta,wd", SHAPES)
@pytest.mark.parametrize("n,batch,pad", [(1, 1, 0), (63, 65, 3), (300, 257, 0), (700, 1000, 24),
                                         (4096, 192, 0)])
def test_shaped_copy_exact(torch, ta, wd, n, batch, pad):
    print_case(test="copy", ta=ta, wd=wd, n=n, batch=batch, pad=pad)
    g = np.random.Generator(np.random.PCG64(n * 7 + batch))
    ld = batch + pad
    src = torch.from_numpy(g.uniform(-1, 1, (n, ld))).cuda()
    dst = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda")
    s_view, d_view = src[:, :batch], dst[:, :batch]
    if (ta, wd) == (1, 4):
        pb.stream_copy(s_view, d_view)
    else:
        pb.stream_copy_shaped(s_view, d_view, ta, wd)
    torch.cuda.synchronize()
    assert torch.equal(dst[:, :batch], src[:, :batch])
    assert bool((dst[:, batch:] == 7.0).all()), "columns past the batch were written"
    before = src.clone()
    pb.stream_copy_shaped(s_view, s_view, ta, wd)
    torch.cuda.synchronize()
    assert torch.equal(src, before)
