"""Pins of the oracle's projection sweep and RK4 step: full-rank agreement with
the brute-force grid step, the closed-form penalty solve, the classical RK4
reduction at mu = 0, energy and divergence identities."""
import numpy as np
import pytest

from oracle import dense as Dn
from oracle import mps as M
from oracle import mpo as O
from oracle import sweep as S
from paper_2406_17823_amd import inputs as I


def test_penalty_fft_matches_explicit_matrix():
    for N in (4, 8):
        dx = 1.0 / N
        rng = np.random.default_rng(N)
        r1, r2 = rng.standard_normal((N, N)), rng.standard_normal((N, N))
        mu, h = 2.5e5, 3e-3
        v1, v2 = Dn.penalty_solve(r1, r2, mu, h, dx)
        A = Dn.penalty_matrix(N, mu, h, dx)
        x = np.linalg.solve(A, np.concatenate([r1.ravel(), r2.ravel()]))
        np.testing.assert_allclose(np.concatenate([v1.ravel(), v2.ravel()]), x, atol=1e-11)


def test_divergence_damped_by_closed_form_factor():
    n = 5
    N, dx = 1 << n, 1.0 / (1 << n)
    rng = np.random.default_rng(1)
    r = (rng.standard_normal((N, N)), rng.standard_normal((N, N)))
    mu, h = 2.5e5, 1e-3
    v = Dn.penalty_solve(r[0], r[1], mu, h, dx)
    kt = Dn.modified_wavenumber(N, dx)
    k2 = kt[:, None] ** 2 + kt[None, :] ** 2
    div_r = np.fft.fft2(Dn.divergence(r, dx))
    div_v = np.fft.fft2(Dn.divergence(v, dx))
    np.testing.assert_allclose(div_v, div_r / (1 + mu * h * h * k2), atol=1e-9 * np.abs(div_r).max())


def test_mu_zero_rk4_is_classical_rk4():
    n = 4
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 4, k0=3.0)
    a = Dn.rk4_step(u, 1e-3, 500.0, 0.0, dx)
    b = Dn.classical_rk4(u, 1e-3, 500.0, dx)
    for i in range(2):
        np.testing.assert_allclose(a[i], b[i], atol=1e-14)


def test_mu_zero_rk1_rk2_are_textbook_euler_and_midpoint():
    """At mu = 0 the minimiser is a - h B(b), so the RK1 / RK2 schedules
    (App. B, Eqs. euler, midpoint_calc, full_calc) must be the textbook
    explicit Euler and midpoint rules."""
    n = 4
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 4, k0=3.0)
    for mine, ref in ((Dn.rk1_step, Dn.classical_euler), (Dn.rk2_step, Dn.classical_midpoint)):
        a = mine(u, 1e-3, 500.0, 0.0, dx)
        b = ref(u, 1e-3, 500.0, dx)
        for i in range(2):
            np.testing.assert_allclose(a[i], b[i], atol=1e-14)


def test_rk1_rk2_observed_order():
    """Global error at a fixed time against a fine RK4 reference halves with
    the step for RK1 and quarters for RK2 (mu = 0: pure time integration)."""
    n = 4
    dx = 1.0 / (1 << n)
    u0 = I.spectrum(n, 4, k0=2.0)
    T, re = 0.04, 200.0

    def run(step, dt):
        u = u0
        for _ in range(int(round(T / dt))):
            u = step(u, dt, re, 0.0, dx)
        return u

    ref = u0
    for _ in range(400):
        ref = Dn.classical_rk4(ref, T / 400, re, dx)

    def err(step, dt):
        u = run(step, dt)
        return float(np.sqrt(sum(np.sum((u[i] - ref[i]) ** 2) for i in range(2))))

    for step, lo, hi in ((Dn.rk1_step, 1.6, 2.4), (Dn.rk2_step, 3.3, 4.7)):
        ratio = err(step, T / 8) / err(step, T / 16)
        assert lo < ratio < hi, (step.__name__, ratio)


def test_skew_symmetric_convection_conserves_energy():
    n = 5
    dx = 1.0 / (1 << n)
    u = I.decaying_jet(n)
    conv = Dn.convection(u[0], u[1], dx)
    s = float(np.sum(u[0] * conv[0] + u[1] * conv[1]))
    scale = float(np.sum(np.abs(u[0] * conv[0]) + np.abs(u[1] * conv[1])))
    assert abs(s) <= 1e-13 * scale


def test_energy_non_increasing_low_re():
    n = 5
    dx = 1.0 / (1 << n)
    u = I.shear_layer(n)
    e0 = Dn.energy(u, dx)
    for _ in range(3):
        u = Dn.rk4_step(u, 1e-3, 1e3, 2.5e5, dx)
        e1 = Dn.energy(u, dx)
        assert e1 <= e0 * (1 + 1e-12)
        e0 = e1


def _mps_of(u, chi):
    return [M.tt_svd(u[i], chi)[0] for i in range(2)]


@pytest.mark.parametrize('mu', [0.0, 2.5e5])
def test_project_full_rank_equals_grid_minimiser(mu):
    n = 3
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 9, k0=2.0)
    b = _mps_of(u, 64)
    a = [M.scale(c, 0.25) for c in b]
    prm = S.Params(re=300.0, dt=1e-3, chi=64, dx=dx, mu=mu, max_sweeps=2)
    h = 2e-3
    v = S.project(a, b, h, prm, a)
    ref = Dn.euler_project((0.25 * u[0], 0.25 * u[1]), u, h, prm.re, mu, dx)
    for i in range(2):
        np.testing.assert_allclose(M.to_dense(v[i]), ref[i], atol=1e-11)


def test_rk4_full_rank_equals_grid_step():
    n = 4
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 2, k0=3.0)
    uc = _mps_of(u, 64)
    u = (M.to_dense(uc[0]), M.to_dense(uc[1]))
    prm = S.Params(re=1e3, dt=1e-3, chi=64, dx=dx, max_sweeps=1)
    new, _ = S.rk4_step(uc, prm)
    ref = Dn.rk4_step(u, prm.dt, prm.re, prm.mu, dx)
    for i in range(2):
        np.testing.assert_allclose(M.to_dense(new[i]), ref[i], atol=1e-11)


@pytest.mark.parametrize('order', [1, 2])
def test_rk1_rk2_full_rank_equal_grid_step(order):
    n = 4
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 2, k0=3.0)
    uc = _mps_of(u, 64)
    u = (M.to_dense(uc[0]), M.to_dense(uc[1]))
    prm = S.Params(re=1e3, dt=1e-3, chi=64, dx=dx, max_sweeps=1)
    new, st = (S.rk1_step if order == 1 else S.rk2_step)(uc, prm)
    assert len(st) == order
    ref = (Dn.rk1_step if order == 1 else Dn.rk2_step)(u, prm.dt, prm.re, prm.mu, dx)
    for i in range(2):
        np.testing.assert_allclose(M.to_dense(new[i]), ref[i], atol=1e-11)


def test_fit_of_B_full_rank_equals_grid_B():
    n = 3
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 9, k0=2.0)
    b = _mps_of(u, 64)
    u = (M.to_dense(b[0]), M.to_dense(b[1]))
    prm = S.Params(re=300.0, dt=1e-3, chi=64, dx=dx, max_sweeps=1)
    w = S.sweep_fit(b, prm, [M.copy(b[0]), M.copy(b[1])])
    ref = Dn.B_field(u[0], u[1], prm.re, dx)
    for i in range(2):
        np.testing.assert_allclose(M.to_dense(w[i]), ref[i], atol=1e-9 * np.abs(ref[i]).max())


def test_explicit_rhs_rk4_full_rank_equals_grid_step():
    n = 4
    dx = 1.0 / (1 << n)
    u = I.spectrum(n, 2, k0=3.0)
    uc = _mps_of(u, 64)
    u = (M.to_dense(uc[0]), M.to_dense(uc[1]))
    prm = S.Params(re=1e3, dt=1e-3, chi=64, dx=dx, max_sweeps=1, rhs_mode=1)
    new, _ = S.rk4_step(uc, prm)
    ref = Dn.rk4_step(u, prm.dt, prm.re, prm.mu, dx)
    for i in range(2):
        np.testing.assert_allclose(M.to_dense(new[i]), ref[i], atol=1e-11)


def test_explicit_rhs_close_to_implicit_when_truncated():
    """Below full rank the fitted B differs from the exact projection by the
    fit's truncation; both minimisers stay close on a smooth flow."""
    n = 5
    dx = 1.0 / (1 << n)
    uc = _mps_of(I.decaying_jet(n), 8)
    a = [M.scale(c, 0.25) for c in uc]
    prm = S.Params(re=1e3, dt=1e-3, chi=8, dx=dx, max_sweeps=2)
    imp = S.project(a, uc, 1e-3 / 6, prm, a)
    prm.rhs_mode = 1
    exp = S.project(a, uc, 1e-3 / 6, prm, a)
    for i in range(2):
        assert M.rel_l2(exp[i], imp[i]) < 1e-3


def _isometry(v, i, d):
    """Dense matrix P_i mapping the centre tensor at site d to the state."""
    n = len(v[i])
    cols = []
    shape = v[i][d].shape
    for e in np.eye(int(np.prod(shape))):
        w = M.copy(v[i])
        w[d] = e.reshape(shape)
        cols.append(M.encode(M.to_dense(w)))
    return np.array(cols).T


def test_local_system_equals_dense_projection():
    """Networks -> local RHS and matrix agree with P^T (a - h B) and
    I + mu h^2 P^T D^T D P formed with explicit isometries (truncated MPS)."""
    n = 3
    N, dx = 1 << n, 1.0 / (1 << n)
    u = I.spectrum(n, 5, k0=2.0)
    b = [M.truncate(x, 3)[0] for x in _mps_of(u, 64)]
    a = [M.scale(x, 0.25) for x in b]
    prm = S.Params(re=200.0, dt=1e-3, chi=3, dx=dx, mu=2.5e5)
    h = 1e-3
    v = [M.right_canonicalize(x) for x in a]
    d = 1
    for i in range(2):
        M.shift_right(v[i], 0)
    rhs_nets, pen = S.build_networks(a, b, h, prm, n)
    for net in rhs_nets + list(pen.values()):
        net.init([M.right_canonicalize(x) for x in a], n)
        net.update_left(v, 0)
    P = [_isometry(v, i, d) for i in range(2)]
    Bd = Dn.B_field(M.to_dense(b[0]), M.to_dense(b[1]), prm.re, dx)
    for i in range(2):
        r = sum(net.coef * net.open(d, net.ket_core(v, d)) for net in rhs_nets if net.bra == i)
        ref = P[i].T @ M.encode(M.to_dense(a[i]) - h * Bd[i])
        np.testing.assert_allclose(r.reshape(-1), ref, atol=1e-12)
    # matrix of the penalty term
    Dm = [O.mpo_to_matrix(O.derivative_mpo(n, ax, 1, dx)) for ax in (1, 2)]
    for i in range(2):
        for j in range(2):
            Kij = P[i].T @ Dm[i].T @ Dm[j] @ P[j]
            shape = v[j][d].shape
            for c in range(Kij.shape[1]):
                e = np.zeros(Kij.shape[1])
                e[c] = 1.0
                col = pen[(i, j)].open(d, e.reshape(shape)).reshape(-1)
                np.testing.assert_allclose(col, Kij[:, c], atol=1e-9)


def test_cg_solves_spd_system():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    A = Q @ np.diag(np.linspace(1, 500, 40)) @ Q.T
    rhs = rng.standard_normal(40)
    x, its, ok = S.cg(lambda z: A @ z, rhs, np.zeros(40), 1e-13, 1000)
    assert ok
    np.testing.assert_allclose(x, np.linalg.solve(A, rhs), rtol=1e-10, atol=1e-12)


def test_theta_not_increased_by_projection():
    """Each local solve is an exact block minimisation of Theta, so the
    projected state is no worse than the guess (truncated MPS)."""
    n = 4
    N, dx = 1 << n, 1.0 / (1 << n)
    u = I.decaying_jet(n)
    b = [M.truncate(x, 6)[0] for x in _mps_of(u, 64)]
    a = [M.scale(x, 0.25) for x in b]
    prm = S.Params(re=1e3, dt=1e-3, chi=6, dx=dx, max_sweeps=2)
    h = 1e-3 / 6
    Bd = Dn.B_field(M.to_dense(b[0]), M.to_dense(b[1]), prm.re, dx)
    Ad = [M.to_dense(x) for x in a]

    def theta(v):
        V = [M.to_dense(x) for x in v]
        div = Dn.divergence(V, dx)
        res = sum(float(np.sum(((V[i] - Ad[i]) / h + Bd[i]) ** 2)) for i in range(2))
        return prm.mu * float(np.sum(div ** 2)) + res

    v = S.project(a, b, h, prm, a)
    assert theta(v) <= theta(a) * (1 + 1e-12)
