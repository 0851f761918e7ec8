"""Seeded synthetic inputs (dense velocity grids and random MPS cores).

This module holds no arithmetic of the solver: it only draws random numbers
and evaluates the closed-form initial conditions on the grid x_m = m / N of
the periodic unit square.  Both the GPU library's tests and the CPU oracle
read their inputs from here.

Flows
-----
shear_layer   double shear layer u = tanh((y - 1/4)/0.02) (y < 1/2),
              tanh((3/4 - y)/0.02) (y >= 1/2), v = 0.05 sin(2 pi x)
decaying_jet  the decaying jet of App. C (jet profile J plus the
              disturbance D, x_min = 0.4, x_max = 0.6, h = 1/200, u0 = 1,
              delta = u0 / (40 A))
spectrum      random-phase field with energy spectrum E(k) (App. C, decaying
              turbulence), divergence-free through a stream function
              differentiated with the central-difference symbol, scaled to
              unit mean kinetic energy
"""
import numpy as np


def grid(n):
    N = 1 << n
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing='ij')
    return X1, X2


def shear_layer(n):
    X1, X2 = grid(n)
    u = np.where(X2 < 0.5, np.tanh((X2 - 0.25) / 0.02), np.tanh((0.75 - X2) / 0.02))
    v = 0.05 * np.sin(2.0 * np.pi * X1)
    return u, v


def decaying_jet(n, x_min=0.4, x_max=0.6, h=1.0 / 200.0, u0=1.0):
    X1, X2 = grid(n)
    J = 0.5 * u0 * (np.tanh((X2 - x_min) / h) - np.tanh((X2 - x_max) / h) - 1.0)
    g_max = np.exp(-((X2 - x_max) ** 2) / h ** 2)
    g_min = np.exp(-((X2 - x_min) ** 2) / h ** 2)
    s = np.sin(8 * np.pi * X1) + np.sin(24 * np.pi * X1) + np.sin(6 * np.pi * X1)
    c = 8 * np.cos(8 * np.pi * X1) + 24 * np.cos(24 * np.pi * X1) + 6 * np.cos(6 * np.pi * X1)
    d1 = 2.0 / h ** 2 * ((X2 - x_max) * g_max + (X2 - x_min) * g_min) * s
    d2 = np.pi * (g_max + g_min) * c
    A = float(np.max(np.sqrt(d1 ** 2 + d2 ** 2)))
    delta = u0 / (40.0 * A)
    return J + delta * d1, delta * d2


def _energy_k4(k, k0):
    return k ** 4 * np.exp(-2.0 * (k / k0) ** 2)


def _energy_paper(k, kp=7.0, s=3):
    a_s = (2 * s + 1) ** (s + 1) / (2 ** s * float(np.prod(np.arange(1, s + 1))))
    return 0.5 * a_s / kp * (k / kp) ** (2 * s + 1) * np.exp(-(s + 0.5) * (k / kp) ** 2)


def spectrum(n, seed, k0=8.0, shape='k4'):
    """Divergence-free random-phase field; shape 'k4' is E ~ k^4 exp(-2 (k/k0)^2),
    shape 'paper' the DT spectrum of App. C (s = 3, k_p = 7)."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(N) * N
    K1, K2 = np.meshgrid(k, k, indexing='ij')
    kk = np.sqrt(K1 ** 2 + K2 ** 2)
    E = _energy_k4(kk, k0) if shape == 'k4' else _energy_paper(kk)
    with np.errstate(divide='ignore', invalid='ignore'):
        amp = np.where(kk > 0, np.sqrt(E / (2.0 * np.pi * np.maximum(kk, 1e-30))) / np.maximum(kk, 1e-30), 0.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(N, N))
    psi_hat = amp * np.exp(1j * phase)
    # symbols of the periodic central difference: i sin(2 pi k / N) * N
    s1 = 1j * np.sin(2.0 * np.pi * K1 / N) * N
    s2 = 1j * np.sin(2.0 * np.pi * K2 / N) * N
    u = np.real(np.fft.ifft2(s2 * psi_hat))
    v = np.real(np.fft.ifft2(-s1 * psi_hat))
    e = 0.5 * float(np.mean(u ** 2 + v ** 2))
    f = 1.0 / np.sqrt(e) if e > 0 else 1.0
    return u * f, v * f


def random_cores(bond_list, seed, scale=1.0):
    """Random MPS cores with the given bonds [1, r_0, ..., 1]; entries
    N(0, scale^2 / (l * 4)) so that the state norm stays O(1)."""
    rng = np.random.default_rng(seed)
    cores = []
    for l, r in zip(bond_list[:-1], bond_list[1:]):
        cores.append(rng.standard_normal((l, 4, r)) * scale / np.sqrt(l * 4.0))
    return cores


def canonical_bonds(n, chi):
    """[1, b_1, ..., b_{n-1}, 1] with b_k = min(chi, 4^k, 4^(n-k))."""
    return [1] + [min(chi, 4 ** k, 4 ** (n - k)) for k in range(1, n)] + [1]


def batch_flows(count=64, base_seed=300):
    """Description of a batch of independent flows of uneven size: flow i has
    n = 8 + (i mod 4), chi = 16 * 2^(floor(i/4) mod 4), a shear layer for
    i < count/2 and a spectrum field otherwise, Re from {1e4, 1e5, 1e6}."""
    out = []
    for i in range(count):
        n = 8 + (i % 4)
        out.append(dict(index=i, n=n, chi=16 * 2 ** ((i // 4) % 4),
                        kind='shear' if i < count // 2 else 'spectrum',
                        re=[1e4, 1e5, 1e6][i % 3], dt=0.2 / (1 << n), seed=base_seed + i))
    return out
