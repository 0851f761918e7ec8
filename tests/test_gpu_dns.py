"""GPU parity of the dense DNS reference (App. D), the fidelity (Eq. fidelity)
and the TKE spectrum (Eqs. TKE) against the oracle, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import dns as S
from paper_2406_17823_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def Q():
    from paper_2406_17823_amd import qtt
    return qtt


@pytest.fixture(scope='module')
def ctx(Q):
    return Q.Context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def field(n, kind, seed=0):
    N = 1 << n
    if kind == 'noise':
        return np.random.default_rng(seed).standard_normal((2, N, N))
    if kind == 'jet':
        return np.asarray(I.decaying_jet(n))
    return np.asarray(S.project(*I.spectrum(n, seed, k0=min(8.0, N / 4))))


@pytest.mark.parametrize('n', [3, 4, 5, 7])
@pytest.mark.parametrize('kind', ['noise', 'spectrum'])
def test_rhs_matches_oracle(Q, ctx, n, kind):
    u = field(n, kind, seed=n)
    re = 1e3
    f = Q.dns_rhs(ctx, dev(u[0]), dev(u[1]), re)
    ref = S.rhs(u[0], u[1], re, 1.0 / (1 << n))
    print(f'[dns] rhs n={n} {kind}', flush=True)
    assert rel(host(f[0]), ref[0]) < 1e-12 and rel(host(f[1]), ref[1]) < 1e-12


@pytest.mark.parametrize('n', [3, 4, 6, 8])
def test_project_matches_oracle(Q, ctx, n):
    u = field(n, 'noise', seed=10 + n)
    g = [dev(u[0]), dev(u[1])]
    Q.dns_project(ctx, g[0], g[1])
    ref = S.project(u[0], u[1])
    print(f'[dns] project n={n}', flush=True)
    assert rel(host(g[0]), ref[0]) < 1e-12 and rel(host(g[1]), ref[1]) < 1e-12
    # idempotent on the GPU too
    h = [x.clone() for x in g]
    Q.dns_project(ctx, h[0], h[1])
    assert rel(host(h[0]), host(g[0])) < 1e-12 and rel(host(h[1]), host(g[1])) < 1e-12


@pytest.mark.parametrize('order', [1, 4])
@pytest.mark.parametrize('n', [3, 6])
def test_step_matches_oracle(Q, ctx, order, n):
    u = field(n, 'spectrum', seed=20 + n)
    re, dt, steps = 500.0, 2e-3, 3
    g = [dev(u[0]), dev(u[1])]
    Q.dns_step(ctx, g[0], g[1], re, dt, order=order, steps=steps)
    ref = S.step([u[0], u[1]], dt, re, 1.0 / (1 << n), order=order, steps=steps)
    print(f'[dns] step n={n} order={order}', flush=True)
    assert rel(host(g[0]), ref[0]) < 1e-11 and rel(host(g[1]), ref[1]) < 1e-11


def test_rk4_step_full_size_jet_matches_oracle(Q, ctx):
    n, re, dt = 11, 1e7, 5e-5
    u = field(n, 'jet')
    g = [dev(u[0]), dev(u[1])]
    print('[dns] rk4 full size jet n=11', flush=True)
    Q.dns_step(ctx, g[0], g[1], re, dt, order=4, steps=1)
    ref = S.rk4_step([u[0], u[1]], dt, re, 1.0 / (1 << n))
    assert rel(host(g[0]), ref[0]) < 1e-11 and rel(host(g[1]), ref[1]) < 1e-11


def test_taylor_green_full_size_closed_form(Q, ctx):
    # explicit diffusion is stable while dt |lap|_max / Re stays inside the
    # RK4 region: about 3e7 dt / Re at 2048 points
    n, re, dt = 11, 1e5, 1e-3
    N = 1 << n
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing='ij')
    u1 = np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X2)
    u2 = -np.cos(2 * np.pi * X1) * np.sin(2 * np.pi * X2)
    lam = -(S.D2_W0 + 2 * sum(w * np.cos(2 * np.pi * m / N)
                                for m, w in enumerate(S.D2_W, start=1))) * N * N
    z = -2.0 * lam * dt / re
    gfac = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** 2
    assert 1 - gfac > 1e-6            # the decay is resolved by the tolerance
    g = [dev(u1), dev(u2)]
    Q.dns_step(ctx, g[0], g[1], re, dt, order=4, steps=2)
    print('[dns] taylor-green n=11', flush=True)
    assert np.abs(host(g[0]) - gfac * u1).max() < 1e-12
    assert np.abs(host(g[1]) - gfac * u2).max() < 1e-12


def test_zero_field_and_zero_steps(Q, ctx):
    N = 1 << 5
    z = [torch.zeros(N, N, dtype=torch.float64, device='cuda') for _ in range(2)]
    Q.dns_step(ctx, z[0], z[1], 10.0, 1e-3, order=4, steps=2)
    assert not bool(z[0].any()) and not bool(z[1].any())
    u = field(5, 'spectrum', seed=3)
    g = [dev(u[0]), dev(u[1])]
    Q.dns_step(ctx, g[0], g[1], 10.0, 1e-3, order=4, steps=0)
    assert np.array_equal(host(g[0]), u[0]) and np.array_equal(host(g[1]), u[1])


@pytest.mark.parametrize('n', [3, 6, 9, 11])
def test_tke_spectrum_matches_oracle(Q, ctx, n):
    u = field(n, 'spectrum' if n < 11 else 'jet', seed=30 + n)
    m = field(n, 'noise', seed=40 + n) * 0.1
    print(f'[dns] tke n={n}', flush=True)
    assert Q.tke_shells(n) == S.shell_count(1 << n)
    E = np.array(Q.tke_spectrum(ctx, dev(u[0]), dev(u[1])))
    ref = S.tke_spectrum(u[0], u[1])
    assert np.abs(E - ref).max() < 1e-12 * ref.max()
    E = np.array(Q.tke_spectrum(ctx, dev(u[0]), dev(u[1]), dev(m[0]), dev(m[1])))
    ref = S.tke_spectrum(u[0], u[1], m[0], m[1])
    assert np.abs(E - ref).max() < 1e-12 * ref.max()


def test_fidelity_matches_oracle(Q, ctx):
    u = field(8, 'spectrum', seed=5)
    v = u + 0.05 * field(8, 'noise', seed=6)
    for i in range(2):
        F = Q.fidelity(ctx, dev(u[i]), dev(v[i]))
        assert F == pytest.approx(S.fidelity(u[i], v[i]), rel=1e-13)
    assert Q.fidelity(ctx, dev(u[0]), dev(-2.5 * u[0])) == pytest.approx(1.0, rel=1e-14)
    z = torch.zeros(16, dtype=torch.float64, device='cuda')
    assert Q.fidelity(ctx, z, dev(np.ones(16))) == 0.0


def test_bad_arguments(Q, ctx):
    g8 = torch.zeros(8, 8, dtype=torch.float64, device='cuda')
    g4 = torch.zeros(4, 4, dtype=torch.float64, device='cuda')
    with pytest.raises(Q.QttError):
        Q.dns_step(ctx, g4, g4.clone(), 10.0, 1e-3)          # n = 2
    with pytest.raises(Q.QttError):
        Q.dns_step(ctx, g8, g8.clone(), 10.0, 1e-3, order=2)
    with pytest.raises(Q.QttError):
        Q.dns_step(ctx, g8, g8.clone(), 0.0, 1e-3)
    with pytest.raises(Q.QttError):
        Q.dns_rhs(ctx, g8, g8, -1.0)
    L = Q.lib()
    E = (ctypes.c_double * Q.tke_shells(3))()
    p = ctypes.c_void_p(g8.data_ptr())
    assert L.qtt_tke_spectrum(ctx.h, p, p, p, None, 3, E, Q.tke_shells(3)) < 0
    assert L.qtt_tke_spectrum(ctx.h, p, p, None, None, 3, E, Q.tke_shells(3) + 1) < 0
    assert Q.tke_shells(2) == 0 and Q.tke_shells(12) == 0
    F = ctypes.c_double()
    assert L.qtt_fidelity(ctx.h, p, p, 0, ctypes.byref(F)) < 0


@pytest.mark.parametrize('n', [6, 8])
def test_results_are_ready_when_the_call_returns(Q, ctx, n):
    # the entry points end with a synchronisation of the library's stream:
    # a read right after the call sees the decayed Taylor-Green field
    N, re, dt = 1 << n, 5e2, 1e-3
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing='ij')
    u1 = np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X2)
    u2 = -np.cos(2 * np.pi * X1) * np.sin(2 * np.pi * X2)
    lam = -(S.D2_W0 + 2 * sum(w * np.cos(2 * np.pi * m / N)
                                for m, w in enumerate(S.D2_W, start=1))) * N * N
    z = -2.0 * lam * dt / re
    g1 = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    for _ in range(3):
        g = [dev(u1), dev(u2)]
        Q.dns_step(ctx, g[0], g[1], re, dt, order=4, steps=1)
        assert np.abs(host(g[0]) - g1 * u1).max() < 1e-13
        f = Q.dns_rhs(ctx, g[0], g[1], re)
        ref = S.rhs(g1 * u1, g1 * u2, re, 1.0 / N)
        assert rel(host(f[0]), ref[0]) < 1e-12 and rel(host(f[1]), ref[1]) < 1e-12
