"""Pins of the oracle's quantics encoding, MPOs and MPS algebra against what
the paper and the mathematics fix (closed forms, brute force on tiny grids,
the Eckart-Young identity of TT-rounding)."""
import os

import numpy as np
import pytest

from oracle import mps as M
from oracle import mpo as O
from paper_2406_17823_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


# ---------------------------------------------------------------- encoding
@pytest.mark.parametrize('n', [1, 2, 3, 5])
def test_encoding_round_trip_bit_exact(n):
    N = 1 << n
    U = np.random.default_rng(n).standard_normal((N, N))
    T = M.encode(U)
    assert np.array_equal(M.decode(T, n), U)
    idx = M.morton_index(n)
    assert sorted(idx.ravel().tolist()) == list(range(N * N))


def test_encoding_x1_is_high_bit():
    # omega_k = (x1^k x2^k)_2 (Sec. II.B): the x1 bit is the high bit of omega
    n = 3
    idx = M.morton_index(n)
    assert idx[4, 0] == 2 * 4 ** 2      # x1 = 100b -> omega_0 = (10)_2
    assert idx[0, 4] == 1 * 4 ** 2      # x2 = 100b -> omega_0 = (01)_2
    assert idx[1, 1] == 3               # last site carries the least significant bits


def test_values_at_equals_dense_field():
    """Pointwise evaluation: the TT-SVD of a dense field is exact at full
    rank, so its values at grid points are the field's; for random cores
    they equal the dense reconstruction's."""
    n = 4
    N = 1 << n
    U = np.random.default_rng(41).standard_normal((N, N))
    cores, _ = M.tt_svd(U, 1 << (2 * n))
    pts = np.random.default_rng(42).integers(0, N, size=(50, 2))
    np.testing.assert_allclose(M.values_at(cores, pts), U[pts[:, 0], pts[:, 1]], rtol=0,
                               atol=1e-12 * np.abs(U).max())
    x = I.random_cores(I.canonical_bonds(n, 7), 43)
    D = M.to_dense(x)
    np.testing.assert_allclose(M.values_at(x, pts), D[pts[:, 0], pts[:, 1]], rtol=0,
                               atol=1e-13 * np.abs(D).max())


# ---------------------------------------------------------------- MPOs
def test_carry_core_matches_paper_table():
    rows = [tuple(int(t) for t in line.split())
            for line in open(os.path.join(GOLDEN, 'diff_mpo_table.txt'))
            if line.strip() and not line.startswith('#')]
    C = O.carry_core(1)
    got = {(a, b, w, v) for a, w, v, b in zip(*np.nonzero(C))}
    assert got == set(rows)
    assert np.all(C[np.nonzero(C)] == 1.0)


def _stencil_matrix(n, axis, weights):
    """Brute force: Morton-ordered matrix of sum_s w_s * (shift by s along axis)."""
    N = 1 << n
    idx = M.morton_index(n)
    A = np.zeros((N * N, N * N))
    for x1 in range(N):
        for x2 in range(N):
            for s, w in weights.items():
                y1, y2 = ((x1 + s) % N, x2) if axis == 1 else (x1, (x2 + s) % N)
                A[idx[x1, x2], idx[y1, y2]] += w
    return A


@pytest.mark.parametrize('n', [1, 2, 3])
@pytest.mark.parametrize('axis', [1, 2])
def test_mpo_equals_brute_force_stencil(n, axis):
    N = 1 << n
    dx = 1.0 / N
    D = O.mpo_to_matrix(O.derivative_mpo(n, axis, 1, dx))
    ref = _stencil_matrix(n, axis, {+1: 1 / (2 * dx), -1: -1 / (2 * dx)})
    np.testing.assert_allclose(D, ref, rtol=0, atol=1e-12 * N)
    D2 = O.mpo_to_matrix(O.derivative_mpo(n, axis, 2, dx))
    ref2 = _stencil_matrix(n, axis, {+1: 1 / dx ** 2, 0: -2 / dx ** 2, -1: 1 / dx ** 2})
    np.testing.assert_allclose(D2, ref2, rtol=0, atol=1e-12 * N * N)
    # central differences are exactly antisymmetric (App. B uses D^T = -D)
    np.testing.assert_array_equal(D.T, -D)


@pytest.mark.parametrize('k', [1, 3, 7])
def test_derivative_of_sines_closed_form(k):
    n = 5
    N = 1 << n
    dx = 1.0 / N
    X1, X2 = I.grid(n)
    th = 2 * np.pi * k * dx
    for axis, X in ((1, X1), (2, X2)):
        x, _ = M.tt_svd(np.sin(2 * np.pi * k * X), 64)
        y = M.to_dense(M.apply_mpo(O.derivative_mpo(n, axis, 1, dx), x))
        np.testing.assert_allclose(y, np.sin(th) / dx * np.cos(2 * np.pi * k * X), atol=1e-11 * N)
        c, _ = M.tt_svd(np.cos(2 * np.pi * k * X), 64)
        y2 = M.to_dense(M.apply_mpo(O.derivative_mpo(n, axis, 2, dx), c))
        np.testing.assert_allclose(y2, -(2 - 2 * np.cos(th)) / dx ** 2 * np.cos(2 * np.pi * k * X),
                                   atol=1e-10 * N * N)
    # literal D o D (lap_mode 1) has the symbol -sin^2(theta)/dx^2
    c, _ = M.tt_svd(np.cos(2 * np.pi * k * X1) + np.cos(2 * np.pi * k * X2), 64)
    y = M.to_dense(M.apply_mpo(O.laplacian_mpo(n, dx, 1), c))
    ref = -np.sin(th) ** 2 / dx ** 2 * (np.cos(2 * np.pi * k * X1) + np.cos(2 * np.pi * k * X2))
    np.testing.assert_allclose(y, ref, atol=1e-10 * N * N)


def test_derivative_of_quadratic_interior():
    # central differences are exact for polynomials of degree <= 2 away from the wrap
    n = 4
    N = 1 << n
    dx = 1.0 / N
    X1, _ = I.grid(n)
    x, _ = M.tt_svd(X1 ** 2, 64)
    y = M.to_dense(M.apply_mpo(O.derivative_mpo(n, 1, 1, dx), x))
    np.testing.assert_allclose(y[1:-1], 2 * X1[1:-1], atol=1e-11)
    y2 = M.to_dense(M.apply_mpo(O.derivative_mpo(n, 1, 2, dx), x))
    np.testing.assert_allclose(y2[1:-1], 2.0 + 0 * X1[1:-1], atol=1e-8)


# ---------------------------------------------------------------- MPS algebra
def _rand(n, chi, seed):
    return I.random_cores(I.canonical_bonds(n, chi), seed)


def test_add_hadamard_apply_dense_and_bonds():
    n = 4
    x, y = _rand(n, 3, 1), _rand(n, 5, 2)
    X, Y = M.to_dense(x), M.to_dense(y)
    s = M.add([2.0, -0.5], [x, y])
    assert M.bonds(s) == [1] + [a + b for a, b in zip(M.bonds(x)[1:-1], M.bonds(y)[1:-1])] + [1]
    np.testing.assert_allclose(M.to_dense(s), 2 * X - 0.5 * Y, atol=1e-13)
    h = M.hadamard(x, y)
    assert M.bonds(h) == [a * b for a, b in zip(M.bonds(x), M.bonds(y))]
    np.testing.assert_allclose(M.to_dense(h), X * Y, atol=1e-13)
    W = O.derivative_mpo(n, 2, 1, 1.0 / 16)
    z = M.apply_mpo(W, x)
    assert M.bonds(z) == [1] + [3 * b for b in M.bonds(x)[1:-1]] + [1]
    np.testing.assert_allclose(M.to_dense(z), (np.roll(X, -1, 1) - np.roll(X, 1, 1)) * 8, atol=1e-12)


def test_hadamard_of_sines():
    n = 5
    X1, _ = I.grid(n)
    s, _ = M.tt_svd(np.sin(2 * np.pi * 3 * X1), 4)
    p = M.hadamard(s, s)
    np.testing.assert_allclose(M.to_dense(p), 0.5 * (1 - np.cos(2 * np.pi * 6 * X1)), atol=1e-13)


def test_tt_svd_full_rank_exact():
    U = np.random.default_rng(5).standard_normal((8, 8))
    x, disc = M.tt_svd(U, 64)
    assert disc < 1e-20
    np.testing.assert_allclose(M.to_dense(x), U, atol=1e-13)
    assert M.bonds(x) == [1, 4, 4, 1]


def _optimal_bond_errors(Y, n, chi):
    """||Y - best rank-chi approximation of unfolding b||^2 for every bond b
    (dense SVD of the quantics unfolding)."""
    T = M.encode(Y)
    out = []
    for k in range(1, n):
        S = np.linalg.svd(T.reshape(4 ** k, -1), compute_uv=False)
        out.append(float(np.sum(S[chi:] ** 2)))
    return out


@pytest.mark.parametrize('chi', [1, 2, 5, 9])
def test_truncate_eckart_young(chi):
    n = 4
    y = M.add([1.0, 0.3, -0.7], [_rand(n, 8, 11), _rand(n, 8, 12), _rand(n, 8, 13)])
    Y = M.to_dense(y)
    t, disc = M.truncate(y, chi)
    T = M.to_dense(t)
    err = float(np.sum((Y - T) ** 2))
    # exact identity of TT-rounding: the error equals the discarded weight
    assert abs(err - disc) <= 1e-12 * max(err, 1e-300) + 1e-26
    eps = _optimal_bond_errors(Y, n, chi)
    assert max(eps) <= err * (1 + 1e-10) + 1e-24
    assert err <= sum(eps) * (1 + 1e-10) + 1e-24
    assert all(b <= min(chi, M.structural_bound(n, k)) for k, b in enumerate(M.bonds(t)))
    # idempotence
    t2, disc2 = M.truncate(t, chi)
    assert disc2 <= 1e-20 * max(1.0, disc)
    np.testing.assert_allclose(M.to_dense(t2), T, atol=1e-12)


def test_truncate_single_bond_is_truncated_svd():
    n = 2
    y = _rand(n, 4, 3)
    Y = M.to_dense(y)
    t, disc = M.truncate(y, 2)
    U, S, Vt = np.linalg.svd(M.encode(Y).reshape(4, 4))
    best = (U[:, :2] * S[:2]) @ Vt[:2]
    np.testing.assert_allclose(M.encode(M.to_dense(t)).reshape(4, 4), best, atol=1e-13)
    assert abs(disc - float(np.sum(S[2:] ** 2))) < 1e-13


def test_truncate_exact_when_chi_covers_rank():
    n = 5
    X1, X2 = I.grid(n)
    U = np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * 3 * X2)     # QTT rank <= 4
    x, _ = M.tt_svd(U, 64)
    y = M.add([1.0, 1.0], [x, x])
    t, disc = M.truncate(y, 4)
    assert disc < 1e-24
    np.testing.assert_allclose(M.to_dense(t), 2 * U, atol=1e-12)


def test_truncate_cutoff_drops_null_directions():
    n = 4
    x = _rand(n, 4, 7)
    y = M.add([0.5, 0.5], [x, x])           # rank of x, bond doubled
    t, _ = M.truncate(y, 64, rtol=1e-12)
    assert M.bonds(t) == M.bonds(M.truncate(x, 64, rtol=1e-12)[0])


def test_rel_l2_and_inner():
    n = 4
    x, y = _rand(n, 4, 1), _rand(n, 4, 2)
    X, Y = M.to_dense(x), M.to_dense(y)
    assert abs(M.inner(x, y) - float(np.sum(X * Y))) < 1e-13
    assert abs(M.rel_l2(x, y) - np.linalg.norm(X - Y) / np.linalg.norm(Y)) < 1e-13
