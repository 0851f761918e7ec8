"""GPU test of the captured CG chunk graphs: RK4 steps whose local CG solves
are replayed from captured graphs give, step after step, bit for bit the
result of the same steps with every kernel launched eagerly (QTT_GRAPHS=0)."""
import numpy as np
import pytest

from oracle import mps as M
from paper_2406_17823_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_graph_replays_equal_eager_launches(monkeypatch):
    from paper_2406_17823_amd import qtt as Q
    n, chi = 7, 32
    u = I.decaying_jet(n)
    uc = [M.tt_svd(u[i], chi, 1e-12)[0] for i in range(2)]
    cap = Q.mps_size(Q.canonical_bonds(n, chi))
    prm = Q.params(re=1e4, dt=0.2 / (1 << n), chi=chi, dx=1.0 / (1 << n), max_sweeps=2)
    monkeypatch.setenv('QTT_GRAPHS', '0')
    eager = Q.Context(0)
    monkeypatch.delenv('QTT_GRAPHS')
    graph = Q.Context(0)
    a = [Q.MPS.from_cores(c, capacity=cap) for c in uc]
    b = [Q.MPS.from_cores(c, capacity=cap) for c in uc]
    replays = 0
    # the graph context's steps alternate with the eager context's (each call
    # synchronises its stream), and every step is compared
    for step in range(4):
        rc, sg = Q.rk4_step(graph, a, prm)
        assert rc == 0
        replays += sg['graph_replays']
        rc, se = Q.rk4_step(eager, b, prm)
        assert rc == 0 and se['graph_replays'] == 0
        assert sg['cg_iters_total'] == se['cg_iters_total'], step
        for i in range(2):
            assert a[i].bonds == b[i].bonds, (step, i)
            for x, y in zip(a[i].cores(), b[i].cores()):
                assert np.array_equal(x, y), (step, i)
    assert replays > 0
    eager.close()
    graph.close()
