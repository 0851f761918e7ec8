"""Pins of the dense DNS oracle (App. D), the fidelity (Eq. fidelity) and the
TKE spectrum (Eqs. TKE) against closed forms and invariants."""
import numpy as np
import pytest

from oracle import dns as S
from paper_2406_17823_amd import inputs as I


def _xy(N):
    x = np.arange(N) / N
    return np.meshgrid(x, x, indexing='ij')


def test_stencils_are_exact_on_polynomials_of_degree_eight():
    # Taylor conditions of an eighth-order central stencil: the first
    # derivative weights reproduce d/dx x^p at 0 for p <= 8, the second
    # derivative weights d^2/dx^2 x^p for p <= 9.
    for p in range(0, 10):
        s1 = sum(w * (m ** p - (-m) ** p) for m, w in enumerate(S.D1_W, start=1))
        s2 = (S.D2_W0 if p == 0 else 0.0) + sum(w * (m ** p + (-m) ** p)
                                                 for m, w in enumerate(S.D2_W, start=1))
        if p <= 8:
            assert s1 == pytest.approx(1.0 if p == 1 else 0.0, abs=1e-13)
        assert s2 == pytest.approx(2.0 if p == 2 else 0.0, abs=1e-12)
    # and not of degree ten: the stencils are exactly eighth order
    assert abs(sum(w * (2 * m ** 9) for m, w in enumerate(S.D1_W, start=1))) > 1.0


def test_derivatives_converge_at_order_eight():
    errs1, errs2 = [], []
    for N in (32, 64):
        X1, X2 = _xy(N)
        U = np.sin(2 * np.pi * X1) * np.cos(4 * np.pi * X2)
        e1 = S.d1(U, 1, 1.0 / N) + 4 * np.pi * np.sin(2 * np.pi * X1) * np.sin(4 * np.pi * X2)
        e2 = S.d2(U, 0, 1.0 / N) + (2 * np.pi) ** 2 * U
        errs1.append(np.abs(e1).max())
        errs2.append(np.abs(e2).max())
    assert 7.5 < np.log2(errs1[0] / errs1[1]) < 8.5
    assert 7.5 < np.log2(errs2[0] / errs2[1]) < 8.5


def test_skew_symmetric_convection_conserves_energy_exactly():
    # Antisymmetric stencils make sum_x u . C vanish for any field.
    rng = np.random.default_rng(3)
    u1, u2 = rng.standard_normal((2, 32, 32))
    c = S.convection(u1, u2, 1.0 / 32)
    scale = np.sum(np.abs(u1 * c[0]) + np.abs(u2 * c[1]))
    assert abs(np.sum(u1 * c[0] + u2 * c[1])) < 1e-13 * scale


def test_convection_of_a_divergence_free_field_is_u_dot_grad_u():
    # psi = sin(2 pi x) sin(4 pi y): u1 = d psi/dy, u2 = -d psi/dx, and
    # (u . grad) u by hand; the skew form converges to it at order eight.
    a, b = 2 * np.pi, 4 * np.pi
    errs = []
    for N in (64, 128):
        X1, X2 = _xy(N)
        u1 = b * np.sin(a * X1) * np.cos(b * X2)
        u2 = -a * np.cos(a * X1) * np.sin(b * X2)
        du1_dx, du1_dy = a * b * np.cos(a * X1) * np.cos(b * X2), -b * b * np.sin(a * X1) * np.sin(b * X2)
        du2_dx, du2_dy = a * a * np.sin(a * X1) * np.sin(b * X2), -a * b * np.cos(a * X1) * np.cos(b * X2)
        c = S.convection(u1, u2, 1.0 / N)
        ex1 = -(u1 * du1_dx + u2 * du1_dy)
        ex2 = -(u1 * du2_dx + u2 * du2_dy)
        errs.append(max(np.abs(c[0] - ex1).max(), np.abs(c[1] - ex2).max()) / np.abs(ex1).max())
    assert errs[0] < 1e-6 and 7.5 < np.log2(errs[0] / errs[1]) < 8.5


def test_projection_properties():
    rng = np.random.default_rng(5)
    N = 32
    u1, u2 = rng.standard_normal((2, N, N))
    p = S.project(u1, u2)
    k = S.projection_wavenumbers(N)
    K1, K2 = np.meshgrid(k, k, indexing='ij')
    div = K1 * np.fft.fft2(p[0]) + K2 * np.fft.fft2(p[1])
    assert np.abs(div).max() < 1e-12 * np.abs(np.fft.fft2(u1)).max()
    # real-symmetric projector: nothing is lost to the real part
    a1 = np.fft.fft2(p[0])
    assert np.abs(a1 - np.conj(np.roll(a1[::-1, ::-1], 1, axis=(0, 1)))).max() < 1e-12
    q = S.project(*p)
    assert np.abs(q[0] - p[0]).max() < 1e-13 and np.abs(q[1] - p[1]).max() < 1e-13
    # a gradient is removed, a curl field kept
    X1, X2 = _xy(N)
    phi_x = 2 * np.pi * np.cos(2 * np.pi * X1) * np.sin(6 * np.pi * X2)
    phi_y = 6 * np.pi * np.sin(2 * np.pi * X1) * np.cos(6 * np.pi * X2)
    g = S.project(phi_x, phi_y)
    assert np.abs(g[0]).max() < 1e-12 and np.abs(g[1]).max() < 1e-12
    c = S.project(phi_y, -phi_x)
    assert np.abs(c[0] - phi_y).max() < 1e-12 and np.abs(c[1] + phi_x).max() < 1e-12
    # the mean flow (kappa = 0) is kept
    m = S.project(np.full((N, N), 0.7), np.full((N, N), -0.2))
    assert np.allclose(m[0], 0.7) and np.allclose(m[1], -0.2)


@pytest.mark.parametrize('order', [1, 4])
def test_taylor_green_decays_at_the_stencil_rate(order):
    # Taylor-Green: the convection is a gradient (projected away) and each
    # velocity component is an eigenvector of the stencil Laplacian with
    # eigenvalue -2 lam, lam = -(w0 + 2 sum w_m cos(2 pi m dx)) / dx^2; one
    # step multiplies the field by the Euler or RK4 polynomial of z.
    N, re, dt = 32, 50.0, 2e-3
    dx = 1.0 / N
    X1, X2 = _xy(N)
    u1 = np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X2)
    u2 = -np.cos(2 * np.pi * X1) * np.sin(2 * np.pi * X2)
    lam = -(S.D2_W0 + 2 * sum(w * np.cos(2 * np.pi * m * dx)
                                for m, w in enumerate(S.D2_W, start=1))) / dx ** 2
    z = -2.0 * lam * dt / re
    g = 1 + z if order == 1 else 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    out = S.step([u1, u2], dt, re, dx, order=order, steps=3)
    assert np.abs(out[0] - g ** 3 * u1).max() < 1e-13
    assert np.abs(out[1] - g ** 3 * u2).max() < 1e-13
    assert abs(lam / (2 * np.pi) ** 2 - 1) < 1e-9    # eighth order at 32 points


@pytest.mark.parametrize('order,expect', [(1, 1.0), (4, 4.0)])
def test_time_order(order, expect):
    n = 5
    N = 1 << n
    u = S.project(*I.spectrum(n, 11, k0=3.0))
    re, T = 100.0, 0.02
    ref = S.step(u, T / 64, re, 1.0 / N, order=order, steps=64)
    e = []
    for k in (2, 4):
        v = S.step(u, T / k, re, 1.0 / N, order=order, steps=k)
        e.append(np.sqrt(np.sum((v[0] - ref[0]) ** 2 + (v[1] - ref[1]) ** 2)))
    assert abs(np.log2(e[0] / e[1]) - expect) < 0.3


def test_projected_step_keeps_the_field_divergence_free_and_zero_stays_zero():
    N = 16
    z = S.step([np.zeros((N, N)), np.zeros((N, N))], 1e-3, 10.0, 1.0 / N)
    assert not np.any(z[0]) and not np.any(z[1])


def test_fidelity():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((16, 16))
    assert S.fidelity(a, -3.0 * a) == pytest.approx(1.0, abs=1e-15)
    X1, _ = _xy(16)
    assert S.fidelity(np.sin(2 * np.pi * X1), np.cos(2 * np.pi * X1)) < 1e-30
    b = a + 0.1 * rng.standard_normal((16, 16))
    cs = np.sum(a * b) ** 2 / (np.sum(a * a) * np.sum(b * b))
    assert 0.9 < S.fidelity(a, b) < 1.0 and S.fidelity(a, b) == pytest.approx(cs, rel=1e-14)


def test_tke_spectrum_single_modes_and_parseval():
    N = 32
    X1, X2 = _xy(N)
    E = S.tke_spectrum(np.sin(2 * np.pi * 3 * X1), np.zeros((N, N)))
    assert E.shape == (S.shell_count(N),) and S.shell_count(N) == 24
    assert E[3] == pytest.approx(0.25, abs=1e-15)      # 1/2 mean(sin^2)
    assert np.abs(np.delete(E, 3)).max() < 1e-30
    E = S.tke_spectrum(np.zeros((N, N)), np.cos(2 * np.pi * (3 * X1 + 4 * X2)))
    assert E[5] == pytest.approx(0.25, abs=1e-15)      # |(3, 4)| = 5
    rng = np.random.default_rng(2)
    u1, u2 = rng.standard_normal((2, N, N))
    m1, m2 = rng.standard_normal((2, N, N))
    E = S.tke_spectrum(u1, u2, m1, m2)
    assert np.sum(E) == pytest.approx(0.5 * np.mean((u1 - m1) ** 2 + (u2 - m2) ** 2), rel=1e-13)
    # a constant mean removes exactly the k = 0 shell
    Ez = S.tke_spectrum(u1, u2, np.full((N, N), u1.mean()), np.full((N, N), u2.mean()))
    assert Ez[0] < 1e-30 and np.allclose(Ez[1:], S.tke_spectrum(u1, u2)[1:], rtol=1e-13)
