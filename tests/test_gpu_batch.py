"""GPU tests of the batched RK4 entry point: independent flows of uneven size
advanced concurrently on worker streams give, flow by flow, exactly the
result of qtt_rk4_step on that flow alone, and one of them matches the
float64 oracle."""
import numpy as np
import pytest

from oracle import mps as M
from oracle import sweep as S
from paper_2406_17823_amd import inputs as I

pytestmark = pytest.mark.gpu

# (flow, n, chi, Re): a small mixed batch in the spirit of the many-flow
# configuration (uneven grids, bonds, Reynolds numbers, both flow families)
FLOWS = [('shear', 5, 8, 1e3), ('jet', 6, 16, 1e4), ('spectrum', 7, 16, 1e5),
         ('spectrum', 5, 4, 1e6), ('jet', 7, 32, 1e5), ('shear', 6, 8, 1e4)]


@pytest.fixture(scope='module')
def Q():
    from paper_2406_17823_amd import qtt
    return qtt


def _flow(kind, n, seed):
    if kind == 'shear':
        return I.shear_layer(n)
    if kind == 'jet':
        return I.decaying_jet(n)
    return I.spectrum(n, seed, k0=4.0)


def _setup(Q, spec, seed):
    kind, n, chi, re = spec
    u = _flow(kind, n, seed)
    uc = [M.tt_svd(u[i], chi, 1e-12)[0] for i in range(2)]
    cap = Q.mps_size(Q.canonical_bonds(n, chi))
    dt = 0.2 / (1 << n)
    prm = Q.params(re=re, dt=dt, chi=chi, dx=1.0 / (1 << n), max_sweeps=1)
    return uc, cap, prm, dt


@pytest.mark.parametrize('workers', [0, 3])
def test_batched_equals_single_flow_calls(Q, workers):
    ctx = Q.Context(0)
    flows, prms, singles = [], [], []
    for f, spec in enumerate(FLOWS):
        uc, cap, prm, _ = _setup(Q, spec, 300 + f)
        flows.append([Q.MPS.from_cores(c, capacity=cap) for c in uc])
        prms.append(prm)
        s = [Q.MPS.from_cores(c, capacity=cap) for c in uc]
        rc, _ = Q.rk4_step(ctx, s, prm)
        assert rc == 0
        singles.append(s)
    rc, stats = Q.rk4_step_batched(ctx, flows, prms, workers)
    assert rc == 0 and len(stats) == len(FLOWS)
    for f in range(len(FLOWS)):
        for i in range(2):
            assert flows[f][i].bonds == singles[f][i].bonds
            a, b = flows[f][i].cores(), singles[f][i].cores()
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (f, i)
        assert stats[f]['cg_solves'] > 0
    ctx.close()


def test_batched_flow_matches_oracle(Q):
    ctx = Q.Context(0)
    specs = [FLOWS[0], FLOWS[3]]
    flows, prms, refs = [], [], []
    for f, spec in enumerate(specs):
        uc, cap, prm, dt = _setup(Q, spec, 400 + f)
        flows.append([Q.MPS.from_cores(c, capacity=cap) for c in uc])
        prms.append(prm)
        kind, n, chi, re = spec
        ref, _ = S.rk4_step(uc, S.Params(re=re, dt=dt, chi=chi, dx=1.0 / (1 << n), max_sweeps=1))
        refs.append(ref)
    rc, _ = Q.rk4_step_batched(ctx, flows, prms, 2)
    assert rc == 0
    for f in range(len(specs)):
        for i in range(2):
            assert flows[f][i].bonds == M.bonds(refs[f][i])
            assert M.rel_l2(flows[f][i].cores(), refs[f][i]) < 1e-10
    ctx.close()


def test_batched_error_names_the_flow(Q):
    ctx = Q.Context(0)
    uc, cap, prm, dt = _setup(Q, FLOWS[0], 500)
    good = [Q.MPS.from_cores(c, capacity=cap) for c in uc]
    # flow 1 asks for chi = 32 with storage only for its current bonds (<= 8)
    short = [Q.MPS.from_cores(c) for c in uc]
    prm_big = Q.params(re=1e3, dt=dt, chi=32, dx=1.0 / 32, max_sweeps=1)
    with pytest.raises(Q.QttError) as e:
        Q.rk4_step_batched(ctx, [good, short], [prm, prm_big], 2)
    assert e.value.code == -3 and 'flow 1' in str(e.value)
    ctx.close()
