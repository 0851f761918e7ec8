"""GPU parity: every entry point of include/qtt.h, called through the C ABI,
against the float64 CPU oracle on identical seeded inputs.

Bars: bond bookkeeping bit-exact; pure data movement and single products
bit-exact; floating-point results within 1e-10 relative L2 (float64 mode).
"""
import numpy as np
import pytest
import torch

from oracle import mpo as O
from oracle import mps as M
from oracle import sweep as S
from paper_2406_17823_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope='module')
def Q():
    from paper_2406_17823_amd import qtt
    return qtt


@pytest.fixture(scope='module')
def ctx(Q):
    return Q.Context(0)


def rand(bonds, seed):
    return I.random_cores(bonds, seed)


def dev(Q, cores, capacity=None):
    return Q.MPS.from_cores(cores, capacity=capacity)


# ---------------------------------------------------------------- data movement / products
def test_add_bit_exact(Q, ctx):
    x = rand([1, 3, 5, 2, 1], 1)
    y = rand([1, 2, 4, 3, 1], 2)
    z = rand([1, 4, 1, 4, 1], 3)
    out = Q.add(ctx, [2.0, -0.5, 0.25], [dev(Q, x), dev(Q, y), dev(Q, z)])
    ref = M.add([2.0, -0.5, 0.25], [x, y, z])
    assert out.bonds == M.bonds(ref)
    for a, b in zip(out.cores(), ref):
        assert np.array_equal(a, b)


def test_add_single_site(Q, ctx):
    x, y = rand([1, 1], 4), rand([1, 1], 5)
    out = Q.add(ctx, [1.5, -1.0], [dev(Q, x), dev(Q, y)])
    np.testing.assert_array_equal(out.cores()[0], M.add([1.5, -1.0], [x, y])[0])


def test_hadamard_bit_exact(Q, ctx):
    a = rand([1, 3, 5, 2, 1], 6)
    b = rand([1, 2, 3, 4, 1], 7)
    out, _ = Q.hadamard(ctx, dev(Q, a), dev(Q, b))
    ref = M.hadamard(a, b)
    assert out.bonds == M.bonds(ref)
    for p, q in zip(out.cores(), ref):
        assert np.array_equal(p, q)


@pytest.mark.parametrize('axis,order', [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_mpo_builder_bit_exact(Q, ctx, axis, order):
    n = 5
    dx = 1.0 / 32
    W = Q.mpo_derivative(ctx, n, axis, order, dx)
    ref = O.derivative_mpo(n, axis, order, dx)
    flat = W.data.cpu().numpy()
    o = 0
    for c in ref:
        assert np.array_equal(flat[o:o + c.size].reshape(c.shape), c)
        o += c.size


def test_apply_mpo_and_sine_derivative(Q, ctx):
    n = 6
    N, dx = 1 << n, 1.0 / (1 << n)
    X1, X2 = I.grid(n)
    x = rand(I.canonical_bonds(n, 5), 8)
    for axis in (1, 2):
        W = Q.mpo_derivative(ctx, n, axis, 1, dx)
        out, _ = Q.apply_mpo(ctx, W, dev(Q, x))
        ref = M.apply_mpo(O.derivative_mpo(n, axis, 1, dx), x)
        assert out.bonds == M.bonds(ref)
        for p, q in zip(out.cores(), ref):
            np.testing.assert_allclose(p, q, rtol=1e-14, atol=1e-14 * np.abs(q).max())
    s, _ = M.tt_svd(np.sin(2 * np.pi * 3 * X2), 64)
    out, _ = Q.apply_mpo(ctx, Q.mpo_derivative(ctx, n, 2, 1, dx), dev(Q, s))
    g = Q.to_dense(ctx, out).cpu().numpy()
    np.testing.assert_allclose(g, np.sin(2 * np.pi * 3 * dx) / dx * np.cos(2 * np.pi * 3 * X2),
                               atol=1e-11 * N)


def test_inner_and_to_dense(Q, ctx):
    n = 7
    x = rand(I.canonical_bonds(n, 12), 9)
    y = rand(I.canonical_bonds(n, 7), 10)
    got = Q.inner(ctx, dev(Q, x), dev(Q, y))
    ref = M.inner(x, y)
    assert abs(got - ref) <= 1e-12 * (abs(ref) + M.norm_sq(x) ** 0.5 * M.norm_sq(y) ** 0.5)
    g = Q.to_dense(ctx, dev(Q, x)).cpu().numpy()
    np.testing.assert_allclose(g, M.to_dense(x), rtol=0, atol=1e-13 * np.abs(M.to_dense(x)).max())


# ---------------------------------------------------------------- truncation
@pytest.mark.parametrize('n,chi,terms,bond,seed', [
    (4, 1, 3, 8, 11), (4, 2, 3, 8, 12), (4, 5, 3, 8, 13), (4, 9, 3, 8, 14),
    (6, 16, 2, 16, 15), (7, 24, 4, 20, 16), (2, 3, 2, 4, 17)])
def test_truncate_matches_oracle(Q, ctx, n, chi, terms, bond, seed):
    xs = [rand(I.canonical_bonds(n, bond), seed * 10 + t) for t in range(terms)]
    coefs = [1.0, 0.3, -0.7, 0.5][:terms]
    y = M.add(coefs, xs)
    ref, disc_ref = M.truncate(y, chi, 1e-12)
    d = dev(Q, y)
    disc = Q.truncate(ctx, d, chi, 1e-12)
    assert d.bonds == M.bonds(ref)
    assert M.rel_l2(d.cores(), ref) < TOL
    assert abs(disc - disc_ref) <= 1e-9 * max(disc_ref, 1e-30) + 1e-28


def test_truncate_ragged_and_rank_cutoff(Q, ctx):
    n = 5
    x = rand([1, 3, 7, 5, 2, 1], 21)
    y = M.add([0.5, 0.5], [x, x])              # doubled bonds, same rank
    d = dev(Q, y)
    Q.truncate(ctx, d, 64, 1e-12)
    ref, _ = M.truncate(y, 64, 1e-12)
    assert d.bonds == M.bonds(ref)
    assert M.rel_l2(d.cores(), x) < TOL


@pytest.mark.parametrize('chi_in,chi', [(37, 48), (37, 20)])
def test_truncate_four_term_sum_blocked_qr(Q, ctx, chi_in, chi):
    """Sum bonds 148 give unfoldings of 256 x 148 and 592 x 148: the blocked
    QR path with four full panels of 32 and a ragged one of 20."""
    n = 8
    xs = [rand(I.canonical_bonds(n, chi_in), 40 + t) for t in range(4)]
    y = M.add([1.0, -0.5, 0.25, 2.0], xs)
    d = dev(Q, y)
    disc = Q.truncate(ctx, d, chi, 1e-12)
    ref, disc_ref = M.truncate(y, chi, 1e-12)
    assert d.bonds == M.bonds(ref)
    assert M.rel_l2(d.cores(), ref) < TOL
    assert abs(disc - disc_ref) <= 1e-9 * max(disc_ref, 1e-30) + 1e-28


def test_truncate_wide_centre_sixteen_slot_gram_rounds(Q, ctx):
    """Four-term sum of bond-150 states on 10 sites: centre bonds of 600 give
    a 600 x 600 Jacobi problem after the QR step (wide unfolding, so V is
    accumulated), too tall for 32 column slots in LDS: the Gram-matrix block
    rounds run with 16 slots over an odd number (75) of 8-column blocks."""
    n = 10
    xs = [rand(I.canonical_bonds(n, 150), 60 + t) for t in range(4)]
    y = M.add([1.0, 0.5, -0.25, 0.75], xs)
    d = dev(Q, y)
    disc = Q.truncate(ctx, d, 200, 1e-12)
    ref, disc_ref = M.truncate(y, 200, 1e-12)
    assert d.bonds == M.bonds(ref)
    assert M.rel_l2(d.cores(), ref) < TOL
    assert abs(disc - disc_ref) <= 1e-9 * max(disc_ref, 1e-30) + 1e-28


# ---------------------------------------------------------------- input compression
def test_from_dense_matches_tt_svd(Q, ctx):
    n, chi = 6, 12
    u = I.decaying_jet(n)
    for comp in range(2):
        g = torch.from_numpy(u[comp]).cuda()
        d = Q.from_dense(ctx, g, chi, 1e-12)
        ref, _ = M.tt_svd(u[comp], chi, 1e-7)
        assert d.bonds == M.bonds(ref)
        # Gram-matrix eigen-decomposition: accurate to ~1e-8 relative
        assert M.rel_l2(d.cores(), ref) < 1e-7


# ---------------------------------------------------------------- projection and RK4
def _mps_pair(u, chi):
    return [M.tt_svd(u[i], chi, 1e-12)[0] for i in range(2)]


def test_project_full_rank_closed_form(Q, ctx):
    from oracle import dense as Dn
    n = 3
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 9, k0=2.0)
    b = _mps_pair(u, 64)
    a = [M.scale(c, 0.25) for c in b]
    prm = Q.params(re=300.0, dt=1e-3, chi=64, dx=dx, max_sweeps=2)
    v = [dev(Q, c) for c in a]
    rc, st = Q.project(ctx, [dev(Q, c) for c in a], [dev(Q, c) for c in b], 2e-3, prm, v)
    assert rc == 0
    ref = Dn.euler_project((0.25 * u[0], 0.25 * u[1]), u, 2e-3, 300.0, 2.5e5, dx)
    for i in range(2):
        np.testing.assert_allclose(M.to_dense(v[i].cores()), ref[i], atol=1e-11)


@pytest.mark.parametrize('flow,n,chi', [('jet', 5, 8), ('spectrum', 5, 8), ('jet', 6, 16)])
def test_project_matches_oracle(Q, ctx, flow, n, chi):
    dx = 1.0 / (1 << n)
    u = I.decaying_jet(n) if flow == 'jet' else I.spectrum(n, 2, k0=4.0)
    b = _mps_pair(u, chi)
    a = [M.scale(c, 0.25) for c in b]
    h = 1e-3 / 3
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2)
    v = [dev(Q, c) for c in a]
    rc, st = Q.project(ctx, [dev(Q, c) for c in a], [dev(Q, c) for c in b], h, prm, v)
    ost = S.Stats()
    ref = S.project(a, b, h, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2), a, ost)
    for i in range(2):
        assert v[i].bonds == M.bonds(ref[i])
        assert M.rel_l2(v[i].cores(), ref[i]) < TOL
    assert abs(st['cg_iters_total'] - ost.cg_iters_total) <= 2 * ost.cg_solves


def test_project_matches_oracle_split_k_matvec(Q, ctx):
    """Bonds [.., 64, 64, 16, ..] make all four penalty-pair GEMMs of the CG
    matvec at site 4 split their K dimension (four reduced outputs in one
    grouped launch)."""
    n, chi = 7, 64
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 2, k0=16.0)
    b = _mps_pair(u, chi)
    a = [M.scale(c, 0.25) for c in b]
    h = 1e-4 / 3
    prm = Q.params(re=1e3, dt=1e-4, chi=chi, dx=dx, max_sweeps=1)
    v = [dev(Q, c) for c in a]
    rc, st = Q.project(ctx, [dev(Q, c) for c in a], [dev(Q, c) for c in b], h, prm, v)
    assert rc == 0
    ref = S.project(a, b, h, S.Params(re=1e3, dt=1e-4, chi=chi, dx=dx, max_sweeps=1), a,
                    S.Stats())
    for i in range(2):
        assert v[i].bonds == M.bonds(ref[i])
        assert M.rel_l2(v[i].cores(), ref[i]) < TOL


def test_project_sweep_stop_rule_matches_oracle(Q, ctx):
    """Sec. II.C stop rule (relative change of sum_i <v_i|v_i> over a full
    sweep at most sweep_rtol): on a case that needs several sweeps the GPU
    stops after the oracle's sweep count with the oracle's state; with the cap
    one sweep below that count it returns QTT_W_SWEEP_MAXIT and the capped
    state."""
    n, chi = 5, 6
    dx = 1.0 / (1 << n)
    u = I.decaying_jet(n)
    b = _mps_pair(u, chi)
    a = [M.scale(c, 0.25) for c in b]
    h = 1e-3 / 3
    ost = S.Stats()
    ref = S.project(a, b, h, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=10,
                                      sweep_rtol=1e-5), a, ost)
    assert ost.sweeps > 1
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=10, sweep_rtol=1e-5)
    v = [dev(Q, c) for c in a]
    rc, st = Q.project(ctx, [dev(Q, c) for c in a], [dev(Q, c) for c in b], h, prm, v)
    assert rc == 0
    assert st['sweeps'][0] == ost.sweeps
    for i in range(2):
        assert v[i].bonds == M.bonds(ref[i])
        assert M.rel_l2(v[i].cores(), ref[i]) < TOL
    cap = ost.sweeps - 1
    ost2 = S.Stats()
    ref2 = S.project(a, b, h, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=cap,
                                       sweep_rtol=1e-5), a, ost2)
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=cap, sweep_rtol=1e-5)
    v = [dev(Q, c) for c in a]
    rc, st = Q.project(ctx, [dev(Q, c) for c in a], [dev(Q, c) for c in b], h, prm, v)
    assert rc == Q.W_SWEEP_MAXIT
    assert st['sweeps'][0] == ost2.sweeps == cap
    for i in range(2):
        assert M.rel_l2(v[i].cores(), ref2[i]) < TOL


def test_project_cg_iteration_limit(Q, ctx):
    """cg_maxit = 3: every local solve stops after three iterations (the CG
    step runs inside the matvec, the limit is tested in its reduction); the
    state, the iteration counts and the warning match the oracle's textbook
    CG stopped at the same iteration."""
    n, chi = 5, 8
    dx = 1.0 / (1 << n)
    u = I.decaying_jet(n)
    b = _mps_pair(u, chi)
    a = [M.scale(c, 0.25) for c in b]
    h = 1e-3 / 3
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2, cg_maxit=3)
    v = [dev(Q, c) for c in a]
    rc, st = Q.project(ctx, [dev(Q, c) for c in a], [dev(Q, c) for c in b], h, prm, v)
    ost = S.Stats()
    ref = S.project(a, b, h, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2,
                                      cg_maxit=3), a, ost)
    assert rc == Q.W_CG_MAXIT
    assert ost.cg_maxit_hits > 0 and st['cg_maxit_hits'] == ost.cg_maxit_hits
    assert st['cg_iters_max'] == 3
    assert st['cg_iters_total'] == ost.cg_iters_total
    for i in range(2):
        assert v[i].bonds == M.bonds(ref[i])
        assert M.rel_l2(v[i].cores(), ref[i]) < TOL


@pytest.mark.parametrize('flow,n,chi', [('shear', 5, 8), ('jet', 5, 8), ('spectrum', 6, 16)])
def test_rk4_matches_oracle(Q, ctx, flow, n, chi):
    dx = 1.0 / (1 << n)
    u = {'shear': I.shear_layer, 'jet': I.decaying_jet}.get(flow, lambda m: I.spectrum(m, 3, 4.0))(n)
    uc = _mps_pair(u, chi)
    cap = Q.mps_size(Q.canonical_bonds(n, chi))
    d = [dev(Q, c, capacity=cap) for c in uc]
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=1)
    rc, st = Q.rk4_step(ctx, d, prm)
    assert rc == 0
    ref, _ = S.rk4_step(uc, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=1))
    for i in range(2):
        assert d[i].bonds == M.bonds(ref[i])
        assert M.rel_l2(d[i].cores(), ref[i]) < TOL


@pytest.mark.parametrize('flow,n,chi,fit', [('jet', 5, 8, 0), ('spectrum', 6, 16, 0),
                                            ('jet', 5, 8, 1)])
def test_project_explicit_rhs_matches_oracle(Q, ctx, flow, n, chi, fit):
    """rhs_mode 1: B(b) fitted as one chi-bounded MPS on the bonds of b, then
    the minimisation with a - h w, against the oracle's same route."""
    dx = 1.0 / (1 << n)
    u = I.decaying_jet(n) if flow == 'jet' else I.spectrum(n, 2, k0=4.0)
    b = _mps_pair(u, chi)
    a = [M.scale(c, 0.25) for c in b]
    h = 1e-3 / 3
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2, rhs_mode=1, fit_sweeps=fit)
    v = [dev(Q, c) for c in a]
    rc, st = Q.project(ctx, [dev(Q, c) for c in a], [dev(Q, c) for c in b], h, prm, v)
    assert rc == 0
    ost = S.Stats()
    ref = S.project(a, b, h, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2,
                                      rhs_mode=1, fit_sweeps=fit), a, ost)
    for i in range(2):
        assert v[i].bonds == M.bonds(ref[i])
        assert M.rel_l2(v[i].cores(), ref[i]) < TOL
    assert st['cg_solves'] == ost.cg_solves
    assert abs(st['cg_iters_total'] - ost.cg_iters_total) <= 2 * ost.cg_solves


def test_rk4_explicit_rhs_matches_oracle(Q, ctx):
    n, chi = 5, 8
    dx = 1.0 / (1 << n)
    uc = _mps_pair(I.shear_layer(n), chi)
    cap = Q.mps_size(Q.canonical_bonds(n, chi))
    d = [dev(Q, c, capacity=cap) for c in uc]
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=1, rhs_mode=1)
    rc, st = Q.rk4_step(ctx, d, prm)
    assert rc == 0
    ref, _ = S.rk4_step(uc, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=1,
                                     rhs_mode=1))
    for i in range(2):
        assert d[i].bonds == M.bonds(ref[i])
        assert M.rel_l2(d[i].cores(), ref[i]) < TOL


@pytest.mark.parametrize('order,flow,n,chi', [(1, 'jet', 5, 8), (2, 'jet', 5, 8),
                                               (1, 'spectrum', 6, 16), (2, 'spectrum', 6, 16)])
def test_rk1_rk2_match_oracle(Q, ctx, order, flow, n, chi):
    """Explicit Euler and midpoint schedules (one and two minimisations from
    the guess u) against the oracle's, through the C ABI."""
    dx = 1.0 / (1 << n)
    u = I.decaying_jet(n) if flow == 'jet' else I.spectrum(n, 3, 4.0)
    uc = _mps_pair(u, chi)
    d = [dev(Q, c) for c in uc]
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2)
    rc, st = Q.rk_step(ctx, d, prm, order)
    assert rc == 0
    step = S.rk1_step if order == 1 else S.rk2_step
    ref, ost = step(uc, S.Params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=2))
    for i in range(2):
        assert d[i].bonds == M.bonds(uc[i]) == M.bonds(ref[i])
        assert M.rel_l2(d[i].cores(), ref[i]) < TOL
    assert st['cg_solves'] == sum(s.cg_solves for s in ost)
    assert abs(st['cg_iters_total'] - sum(s.cg_iters_total for s in ost)) <= \
        2 * st['cg_solves']


def test_rk_step_order_four_is_rk4_step(Q, ctx):
    n, chi = 5, 8
    dx = 1.0 / (1 << n)
    uc = _mps_pair(I.shear_layer(n), chi)
    cap = Q.mps_size(Q.canonical_bonds(n, chi))
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=dx, max_sweeps=1)
    d1 = [dev(Q, c, capacity=cap) for c in uc]
    d2 = [dev(Q, c, capacity=cap) for c in uc]
    assert Q.rk4_step(ctx, d1, prm)[0] == 0
    assert Q.rk_step(ctx, d2, prm, 4)[0] == 0
    for i in range(2):
        assert d1[i].bonds == d2[i].bonds
        assert np.array_equal(np.concatenate([c.ravel() for c in d1[i].cores()]),
                              np.concatenate([c.ravel() for c in d2[i].cores()]))


# ---------------------------------------------------------------- error paths
def test_rk_step_bad_order(Q, ctx):
    n, chi = 4, 4
    uc = _mps_pair(I.shear_layer(n), chi)
    d = [dev(Q, c) for c in uc]
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=1.0 / (1 << n))
    with pytest.raises(Q.QttError) as e:
        Q.rk_step(ctx, d, prm, 3)
    assert e.value.code == -1  # QTT_E_ARG


def test_bad_rhs_mode(Q, ctx):
    n, chi = 4, 4
    uc = _mps_pair(I.shear_layer(n), chi)
    d = [dev(Q, c) for c in uc]
    prm = Q.params(re=1e3, dt=1e-3, chi=chi, dx=1.0 / (1 << n), rhs_mode=2)
    with pytest.raises(Q.QttError) as e:
        Q.project(ctx, d, d, 1e-3, prm, [dev(Q, c) for c in uc])
    assert e.value.code == -1  # QTT_E_ARG


def test_capacity_error(Q, ctx):
    x = rand([1, 4, 4, 1], 30)
    y = Q.MPS.empty([1, 1, 1, 1], capacity=4)
    with pytest.raises(Q.QttError) as e:
        Q.add(ctx, [1.0, 1.0], [dev(Q, x), dev(Q, x)], y)
    assert e.value.code == -3


def test_nan_input_rejected(Q, ctx):
    n = 3
    x = rand(I.canonical_bonds(n, 4), 31)
    x[1][0, 0, 0] = np.nan
    a = [dev(Q, x), dev(Q, rand(I.canonical_bonds(n, 4), 32))]
    prm = Q.params(re=1e3, dt=1e-3, chi=4, dx=1 / 8)
    with pytest.raises(Q.QttError) as e:
        Q.project(ctx, a, a, 1e-3, prm, [dev(Q, c.cores()) for c in a])
    assert e.value.code == -5


def test_svd_sweep_cap_warns(Q, monkeypatch):
    """A Jacobi SVD stopped at its sweep cap with rotations pending makes the
    call return QTT_W_SVD_MAXIT (the cap forced to one sweep from the host);
    at the default cap the same truncation converges and returns 0."""
    n = 9   # sum bonds 160 at sites 4, 5: blocked Jacobi with several outer sweeps
    xs = [rand(I.canonical_bonds(n, 40), 90 + t) for t in range(4)]
    y = M.add([1.0, 0.3, -0.7, 0.5], xs)
    monkeypatch.setenv('QTT_SVD_MAX_SWEEPS', '1')
    capped = Q.Context(0)
    monkeypatch.delenv('QTT_SVD_MAX_SWEEPS')
    d = dev(Q, y)
    Q.truncate(capped, d, 48, 1e-12)
    assert capped.last_warning == Q.W_SVD_MAXIT
    capped.close()
    normal = Q.Context(0)
    d = dev(Q, y)
    Q.truncate(normal, d, 48, 1e-12)
    assert normal.last_warning == 0
    ref, _ = M.truncate(y, 48, 1e-12)
    assert M.rel_l2(d.cores(), ref) < TOL
    normal.close()
