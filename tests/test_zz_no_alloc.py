"""The allocation-free inner product (qtt_inner_noalloc) through the C ABI
against qtt_inner on the same inputs: two calls in a row, the second with
smaller bonds, plus the size limit and argument errors."""
import numpy as np
import pytest
import torch

from paper_2406_17823_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def Q():
    from paper_2406_17823_amd import qtt
    return qtt


def _pair(Q, n, bx, by, seed):
    x = Q.MPS.from_cores(I.random_cores(I.canonical_bonds(n, bx), seed))
    y = Q.MPS.from_cores(I.random_cores(I.canonical_bonds(n, by), seed + 1))
    return x, y


def test_inner_noalloc_matches_inner_twice(Q):
    ctx = Q.Context(0)
    out = torch.full((1,), np.nan, dtype=torch.float64, device='cuda')
    for n, bx, by, seed in ((11, 128, 128, 70), (6, 16, 9, 72)):
        x, y = _pair(Q, n, bx, by, seed)
        ref = Q.inner(ctx, x, y)
        rc = Q.inner_noalloc(x, y, out)
        torch.cuda.synchronize()
        assert rc == 0
        got = float(out.item())
        scale = (Q.inner(ctx, x, x) * Q.inner(ctx, y, y)) ** 0.5
        assert abs(got - ref) <= 1e-12 * scale, (n, got, ref)
    ctx.close()


def test_inner_noalloc_limits(Q):
    out = torch.zeros(1, dtype=torch.float64, device='cuda')
    x, y = _pair(Q, 10, 300, 300, 74)    # 300 * 300 > 65536
    assert Q.inner_noalloc(x, y, out) == -3
    x, y = _pair(Q, 5, 8, 8, 76)
    z = Q.MPS.from_cores(I.random_cores(I.canonical_bonds(4, 8), 78))
    assert Q.inner_noalloc(x, z, out) == -1
    torch.cuda.synchronize()
