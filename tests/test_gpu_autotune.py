"""The GEMM tile autotuner changes only speed: a context that tunes tile sizes
and one that keeps the heuristic choice produce bitwise identical RK4 steps
(split-K is decided on the 64 x 64 tiling, so the summation order is the
same for every tile size)."""
import os

import numpy as np
import pytest

from oracle import mps as M
from paper_2406_17823_amd import inputs as I

pytestmark = pytest.mark.gpu


def _step(Q, tune, n, chi):
    os.environ['QTT_AUTOTUNE'] = '1' if tune else '0'  # read when the context is created
    try:
        ctx = Q.Context(0)
    finally:
        os.environ.pop('QTT_AUTOTUNE')
    u = I.spectrum(n, 7, k0=8.0)
    uc = [M.tt_svd(u[i], chi, 1e-12)[0] for i in range(2)]
    cap = Q.mps_size(Q.canonical_bonds(n, chi))
    d = [Q.MPS.from_cores(c, capacity=cap) for c in uc]
    prm = Q.params(re=1e5, dt=2e-4, chi=chi, dx=1.0 / (1 << n), max_sweeps=1,
                   prec=Q.PREC_F64)
    rc, _ = Q.rk4_step(ctx, d, prm)
    assert rc == 0
    out = [x.cores() for x in d]
    ctx.close()
    return out


def test_autotuned_tiles_give_identical_results():
    from paper_2406_17823_amd import qtt as Q
    n, chi = 8, 64
    a = _step(Q, True, n, chi)
    b = _step(Q, False, n, chi)
    for i in range(2):
        assert len(a[i]) == len(b[i])
        for x, y in zip(a[i], b[i]):
            assert x.shape == y.shape and np.array_equal(x, y)
