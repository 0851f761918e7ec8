"""Dense direct numerical simulation (DNS) reference, fidelity and TKE spectrum
-- test oracle (see package docstring).

The paper verifies its tensor-network solver against a grid DNS (App. D)
and compares the two by the fidelity (Eq. fidelity) and the turbulent
kinetic energy spectrum (Eqs. TKE).  This module writes those definitions
out on the periodic unit square, N x N points, U[i1, i2] = u(i1 dx, i2 dx):

  * first and second derivatives by the eighth-order central stencils
    (Fornberg's weights for offsets 1..4), periodic;
  * skew-symmetric convection C_i = -1/2 sum_j (u_j d_j u_i + d_j(u_j u_i))
    and diffusion D_i = (1/Re) (d_11 + d_22) u_i;
  * the projection onto divergence-free fields in Fourier space,
    u^ - kappa (kappa . u^) / |kappa|^2 for kappa != 0 (Eq. projection),
    with the Nyquist component of kappa taken as 0, followed by the real
    part of the inverse transform (a no-op up to rounding);
  * the explicit Euler step u <- P(u + dt (C + D)) and its RK4 extension,
    in which every stage velocity and the final combination are projected;
  * F = |<a|b>|^2 / (||a||^2 ||b||^2) per component;
  * E(k1, k2) = 1/2 (|u1'^|^2 + |u2'^|^2) with u^ = FFT(u - mean) / N^2 and
    E(k) the sum over the integer shell round(|kappa|) = k, kappa in units
    of 2 pi (integer wavenumbers).
"""
import numpy as np

# Eighth-order central weights (Fornberg, "Generation of finite difference
# formulas on arbitrarily spaced grids", 1988): offsets 1..4.
D1_W = (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0)
D2_W0 = -205.0 / 72.0
D2_W = (8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)


def d1(U, axis, dx):
    """sum_m w_m (U[x+m] - U[x-m]) / dx, periodic."""
    out = np.zeros_like(U)
    for m, w in enumerate(D1_W, start=1):
        out += w * (np.roll(U, -m, axis=axis) - np.roll(U, m, axis=axis))
    return out / dx


def d2(U, axis, dx):
    """(w_0 U + sum_m w_m (U[x+m] + U[x-m])) / dx^2, periodic."""
    out = D2_W0 * U
    for m, w in enumerate(D2_W, start=1):
        out = out + w * (np.roll(U, -m, axis=axis) + np.roll(U, m, axis=axis))
    return out / (dx * dx)


def convection(u1, u2, dx):
    """Skew-symmetric convection C_i = -1/2 sum_j (u_j d_j u_i + d_j(u_j u_i))."""
    u = (u1, u2)
    out = []
    for i in range(2):
        c = np.zeros_like(u1)
        for j in range(2):
            c -= 0.5 * (u[j] * d1(u[i], j, dx) + d1(u[j] * u[i], j, dx))
        out.append(c)
    return out


def diffusion(u1, u2, re, dx):
    return [(d2(u, 0, dx) + d2(u, 1, dx)) / re for u in (u1, u2)]


def rhs(u1, u2, re, dx):
    """C + D of the momentum equation without the pressure term."""
    c = convection(u1, u2, dx)
    d = diffusion(u1, u2, re, dx)
    return [c[0] + d[0], c[1] + d[1]]


def wavenumbers(N):
    """Integer wavenumbers in FFT order (the Nyquist index as -N/2)."""
    return np.fft.fftfreq(N) * N


def projection_wavenumbers(N):
    """Wavenumbers of the projection: the Nyquist component taken as 0 (the
    odd-derivative convention), so that the projector at k and -k agree and
    a real field stays real."""
    k = wavenumbers(N)
    k[N // 2] = 0.0
    return k


def project(u1, u2):
    """Divergence-free part: u^ - kappa (kappa . u^)/|kappa|^2, kappa != 0."""
    N = u1.shape[0]
    k = projection_wavenumbers(N)
    K1, K2 = np.meshgrid(k, k, indexing='ij')
    a1, a2 = np.fft.fft2(u1), np.fft.fft2(u2)
    k2 = K1 * K1 + K2 * K2
    k2[k2 == 0.0] = 1.0
    s = (K1 * a1 + K2 * a2) / k2
    return [np.real(np.fft.ifft2(a1 - K1 * s)), np.real(np.fft.ifft2(a2 - K2 * s))]


def euler_step(u, dt, re, dx):
    """Explicit Euler with projection: u* = u + dt (C + D), u <- P(u*)."""
    f = rhs(u[0], u[1], re, dx)
    return project(u[0] + dt * f[0], u[1] + dt * f[1])


def rk4_step(u, dt, re, dx):
    """Classical RK4 on du/dt = C + D, every stage velocity projected."""
    f1 = rhs(u[0], u[1], re, dx)
    w2 = project(u[0] + 0.5 * dt * f1[0], u[1] + 0.5 * dt * f1[1])
    f2 = rhs(w2[0], w2[1], re, dx)
    w3 = project(u[0] + 0.5 * dt * f2[0], u[1] + 0.5 * dt * f2[1])
    f3 = rhs(w3[0], w3[1], re, dx)
    w4 = project(u[0] + dt * f3[0], u[1] + dt * f3[1])
    f4 = rhs(w4[0], w4[1], re, dx)
    return project(*[u[i] + dt / 6.0 * (f1[i] + 2.0 * f2[i] + 2.0 * f3[i] + f4[i])
                     for i in range(2)])


def step(u, dt, re, dx, order=4, steps=1):
    for _ in range(steps):
        u = rk4_step(u, dt, re, dx) if order == 4 else euler_step(u, dt, re, dx)
    return u


def fidelity(a, b):
    """|<a|b>|^2 / (||a||^2 ||b||^2) (Eq. fidelity)."""
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.dot(a, b) ** 2 / (np.dot(a, a) * np.dot(b, b)))


def shell_count(N):
    """Number of integer shells k = 0 .. round(sqrt(2) N/2)."""
    return int(np.rint(np.sqrt(2.0) * (N // 2))) + 1


def tke_spectrum(u1, u2, mean1=None, mean2=None):
    """E(k), k = 0 .. shell_count(N) - 1 (Eqs. TKE, shell sum)."""
    N = u1.shape[0]
    f1 = u1 - (0.0 if mean1 is None else mean1)
    f2 = u2 - (0.0 if mean2 is None else mean2)
    a1 = np.fft.fft2(f1) / (N * N)
    a2 = np.fft.fft2(f2) / (N * N)
    E2 = 0.5 * (np.abs(a1) ** 2 + np.abs(a2) ** 2)
    k = wavenumbers(N)
    K1, K2 = np.meshgrid(k, k, indexing='ij')
    shell = np.rint(np.sqrt(K1 * K1 + K2 * K2)).astype(np.int64)
    E = np.zeros(shell_count(N))
    np.add.at(E, shell.ravel(), E2.ravel())
    return E
