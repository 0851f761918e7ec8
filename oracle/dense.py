"""Brute-force full-grid step -- test oracle (see package docstring).

The QTT step computes, at full bond dimension, exactly what this module
computes on the N x N grid:

  * periodic central differences D_j (Eq. fdm) and three-point D_j^2;
  * B_i(b) = sum_j 1/2 (b_j D_j b_i + D_j (b_j b_i)) - (1/Re) D_j^2 b_i
    (App. B, skew-symmetric convection of Eq. MPS_momentum, explicit
    diffusion);
  * the minimiser of Theta (App. B, Eq. Theta) over all grid fields:
    (I + mu h^2 D^T D) v = a - h B(b), D v = D_1 v_1 + D_2 v_2, solved
    per Fourier mode in closed form (D_j is circulant);
  * RK4 as four Euler minimisations with the b-table (App. B, Table RK4,
    Eqs. U1-U4); RK1 as one minimisation and RK2 as the midpoint pair of
    minimisations (App. B, Eqs. euler, midpoint_calc, full_calc).
"""
import numpy as np


def d1(U, axis, dx):
    """(U[x+1] - U[x-1]) / (2 dx) along one axis, periodic."""
    return (np.roll(U, -1, axis=axis) - np.roll(U, 1, axis=axis)) / (2.0 * dx)


def d2(U, axis, dx, lap_mode=0):
    """Second difference: three-point (lap_mode 0) or D o D (lap_mode 1)."""
    if lap_mode == 1:
        return d1(d1(U, axis, dx), axis, dx)
    return (np.roll(U, -1, axis=axis) - 2.0 * U + np.roll(U, 1, axis=axis)) / (dx * dx)


def convection(b1, b2, dx):
    """sum_j 1/2 (b_j D_j b_i + D_j(b_j b_i)) for i = 1, 2."""
    b = (b1, b2)
    out = []
    for i in range(2):
        c = np.zeros_like(b1)
        for j in range(2):
            c += 0.5 * (b[j] * d1(b[i], j, dx) + d1(b[j] * b[i], j, dx))
        out.append(c)
    return out


def B_field(b1, b2, re, dx, lap_mode=0):
    """B_i(b) of App. B (the negative right-hand side of the momentum eq.)."""
    conv = convection(b1, b2, dx)
    b = (b1, b2)
    return [conv[i] - (d2(b[i], 0, dx, lap_mode) + d2(b[i], 1, dx, lap_mode)) / re
            for i in range(2)]


def modified_wavenumber(N, dx):
    """Eigenvalue of the central difference on exp(2 pi i k x): i*sin(2 pi k dx)/dx."""
    k = np.fft.fftfreq(N) * N
    return np.sin(2.0 * np.pi * k * dx) / dx


def penalty_solve(r1, r2, mu, h, dx):
    """Solve (I + mu h^2 D^T D) v = r on the grid, per Fourier mode:
    v^ = r^ - mu h^2 kt (kt . r^) / (1 + mu h^2 |kt|^2) (Sherman-Morrison)."""
    N = r1.shape[0]
    kt = modified_wavenumber(N, dx)
    K1 = kt[:, None] * np.ones((1, N))
    K2 = np.ones((N, 1)) * kt[None, :]
    R1 = np.fft.fft2(r1)
    R2 = np.fft.fft2(r2)
    g = mu * h * h
    dot = K1 * R1 + K2 * R2
    den = 1.0 + g * (K1 * K1 + K2 * K2)
    V1 = R1 - g * K1 * dot / den
    V2 = R2 - g * K2 * dot / den
    return np.real(np.fft.ifft2(V1)), np.real(np.fft.ifft2(V2))


def penalty_matrix(N, mu, h, dx):
    """The explicit (2N^2 x 2N^2) matrix I + mu h^2 D^T D (tiny N only);
    unknowns ordered (component, x1, x2)."""
    M = N * N
    D = [np.zeros((M, M)), np.zeros((M, M))]
    for x1 in range(N):
        for x2 in range(N):
            row = x1 * N + x2
            D[0][row, ((x1 + 1) % N) * N + x2] += 1.0 / (2 * dx)
            D[0][row, ((x1 - 1) % N) * N + x2] -= 1.0 / (2 * dx)
            D[1][row, x1 * N + (x2 + 1) % N] += 1.0 / (2 * dx)
            D[1][row, x1 * N + (x2 - 1) % N] -= 1.0 / (2 * dx)
    Dfull = np.hstack(D)
    return np.eye(2 * M) + mu * h * h * Dfull.T @ Dfull


def euler_project(a, b, h, re, mu, dx, lap_mode=0):
    """argmin over grid fields of Theta(v, a, b, h)."""
    B = B_field(b[0], b[1], re, dx, lap_mode)
    return penalty_solve(a[0] - h * B[0], a[1] - h * B[1], mu, h, dx)


RK4_B_TABLE = [(3.0, 0.25), (1.5, 0.625), (3.0, 0.25)]
RK4_H = [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]


def rk4_step(u, dt, re, mu, dx, lap_mode=0):
    """One RK4 step as four Euler minimisations (App. B, Eqs. U1-U4)."""
    a = (0.25 * u[0], 0.25 * u[1])
    U = []
    for k in range(4):
        if k == 0:
            b = u
        else:
            c, cu = RK4_B_TABLE[k - 1]
            b = (c * U[-1][0] + cu * u[0], c * U[-1][1] + cu * u[1])
        U.append(euler_project(a, b, RK4_H[k] * dt, re, mu, dx, lap_mode))
    return (sum(x[0] for x in U), sum(x[1] for x in U))


def rk1_step(u, dt, re, mu, dx, lap_mode=0):
    """Explicit Euler as one minimisation (App. B, Eq. euler): a = b = u."""
    return euler_project(u, u, dt, re, mu, dx, lap_mode)


def rk2_step(u, dt, re, mu, dx, lap_mode=0):
    """Midpoint RK2 as two minimisations (App. B, Eqs. midpoint_calc,
    full_calc): u_mid from (a, b, h) = (u, u, dt/2), then (u, u_mid, dt)."""
    mid = euler_project(u, u, 0.5 * dt, re, mu, dx, lap_mode)
    return euler_project(u, mid, dt, re, mu, dx, lap_mode)


def classical_euler(u, dt, re, dx, lap_mode=0):
    """Textbook explicit Euler on du/dt = -B(u) (no penalty)."""
    B = B_field(u[0], u[1], re, dx, lap_mode)
    return (u[0] - dt * B[0], u[1] - dt * B[1])


def classical_midpoint(u, dt, re, dx, lap_mode=0):
    """Textbook explicit midpoint rule on du/dt = -B(u) (no penalty)."""
    B = B_field(u[0], u[1], re, dx, lap_mode)
    m = (u[0] - 0.5 * dt * B[0], u[1] - 0.5 * dt * B[1])
    Bm = B_field(m[0], m[1], re, dx, lap_mode)
    return (u[0] - dt * Bm[0], u[1] - dt * Bm[1])


def classical_rk4(u, dt, re, dx, lap_mode=0):
    """Textbook RK4 on du/dt = -B(u) (no penalty), for pinning the b-table."""
    def f(v):
        B = B_field(v[0], v[1], re, dx, lap_mode)
        return (-B[0], -B[1])
    k1 = f(u)
    k2 = f((u[0] + 0.5 * dt * k1[0], u[1] + 0.5 * dt * k1[1]))
    k3 = f((u[0] + 0.5 * dt * k2[0], u[1] + 0.5 * dt * k2[1]))
    k4 = f((u[0] + dt * k3[0], u[1] + dt * k3[1]))
    return tuple(u[i] + dt / 6.0 * (k1[i] + 2 * k2[i] + 2 * k3[i] + k4[i]) for i in range(2))


def energy(u, dx):
    return 0.5 * float(np.sum(u[0] ** 2 + u[1] ** 2)) * dx * dx


def divergence(u, dx):
    return d1(u[0], 0, dx) + d1(u[1], 1, dx)
