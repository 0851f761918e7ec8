"""What a block-diagonal preconditioner of the local penalty solves can gain
(the learned preconditioner's feature blocks are the diagonal blocks of one
velocity component, chi * 4 * chi, or smaller).  Parity unpinned: none;
these are properties of the oracle's local matrices.

Full rank (the local trial space is the whole grid): the local matrix is
unitarily equivalent to I + mu h^2 D^T D (App. B, Eq. big_LS), which the
Fourier modes block-diagonalise into 2 x 2 blocks
    [[1 + a, s_ab], [s_ab, 1 + b]],  a = c k1~^2, b = c k2~^2, |s_ab| = sqrt(a b),
with c = mu h^2 and kj~ = sin(2 pi kj dx) / dx.  The exact inverse of the two
component blocks turns each into [[1, x], [y, 1]] with eigenvalues
1 +- sqrt(a b / ((1 + a)(1 + b))), so on the diagonal wave vector k1 = k2 =
N/4 the preconditioned condition number is 1 + 2 c / dx^2, the unpreconditioned
one: the exact component-block inverse leaves the condition number unchanged
(and for a 2 x 2 block no diagonal scaling does better than the one that
equalises its diagonal).

Truncated (chi below full rank): on an actual local system of a sweep the
exact inverse of the 4 x 4 position blocks (the network's block form) does
not lower the CG iteration count, and neither do the two structured
approximations of a whole component block that could be applied at
O(chi^3) cost (a Kronecker sum L + W + R or a Kronecker product L x W x R of
chi x chi, 4 x 4 and chi x chi factors, each the Frobenius-nearest of its
form) over the local solves of a sweep.
"""
import numpy as np

from oracle import mps as M
from oracle import sweep as S
from paper_2406_17823_amd import inputs as I


def _local_matrix(a, b, h, prm, d):
    """Dense local matrix of the penalty solve at centre d (the CG operator of
    the one-site sweep), the stacked local right-hand side and the current
    centre, built with the oracle's networks."""
    n = len(a[0])
    v = [M.right_canonicalize(x) for x in a]
    rhs_nets, pen = S.build_networks(a, b, h, prm, n)
    for net in rhs_nets + list(pen.values()):
        net.init(v, n)
    for k in range(d):
        for i in range(2):
            M.shift_right(v[i], k)
        for net in rhs_nets + list(pen.values()):
            net.update_left(v, k)
    shape = [v[i][d].shape for i in range(2)]
    sizes = [int(np.prod(s)) for s in shape]
    N = sum(sizes)
    A = np.zeros((N, N))
    for col in range(N):
        e = np.zeros(N)
        e[col] = 1.0
        xs = [e[:sizes[0]].reshape(shape[0]), e[sizes[0]:].reshape(shape[1])]
        y = [xs[0].copy(), xs[1].copy()]
        for (i, j), net in pen.items():
            y[i] = y[i] + net.coef * net.open(d, xs[j])
        A[:, col] = np.concatenate([y[0].ravel(), y[1].ravel()])
    r = []
    for i in range(2):
        t = np.zeros(shape[i])
        for net in rhs_nets:
            if net.bra == i:
                t += net.coef * net.open(d, net.ket_core(v, d))
        r.append(t.ravel())
    x0 = np.concatenate([v[0][d].ravel(), v[1][d].ravel()])
    return 0.5 * (A + A.T), np.concatenate(r), x0, sizes[0], shape


def _comp_block_precond(A, n0):
    B1 = np.linalg.inv(A[:n0, :n0])
    B2 = np.linalg.inv(A[n0:, n0:])
    return lambda r: np.concatenate([B1 @ r[:n0], B2 @ r[n0:]]), B1, B2


def _pcg_iters(A, rhs, x0, Minv, rtol=1e-10, maxit=10000):
    x = x0.copy()
    r = rhs - A @ x
    bn = np.linalg.norm(rhs)
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = A @ p
        al = rz / (p @ q)
        x += al * p
        r -= al * q
        if np.linalg.norm(r) <= rtol * bn:
            return it
        z = Minv(r)
        rz2 = r @ z
        p = z + (rz2 / rz) * p
        rz = rz2
    return maxit


def test_component_block_inverse_keeps_condition_number_full_rank():
    n = 4
    N, dx = 1 << n, 1.0 / (1 << n)
    u = I.spectrum(n, 4, k0=2.0)
    b = [M.tt_svd(u[i], 64, 1e-14)[0] for i in range(2)]
    assert [M.bonds(x) for x in b] == [[1, 4, 16, 4, 1]] * 2       # full rank
    a = [M.scale(x, 0.25) for x in b]
    h = 2e-3
    prm = S.Params(re=1e3, dt=3 * h, chi=64, dx=dx)
    A, rhs, x0, n0, _ = _local_matrix(a, b, h, prm, 1)
    assert A.shape == (2 * N * N, 2 * N * N)
    c = prm.mu * h * h
    k = np.arange(N)
    kt = np.sin(2 * np.pi * k * dx) / dx
    aa = c * kt[:, None] ** 2 * np.ones((1, N))
    bb = c * np.ones((N, 1)) * kt[None, :] ** 2
    # spectrum of A: 1 (divergence-free part) and 1 + a + b per mode
    ev = np.linalg.eigvalsh(A)
    ref = np.sort(np.concatenate([np.ones(N * N), (1 + aa + bb).ravel()]))
    np.testing.assert_allclose(ev, ref, rtol=1e-10, atol=1e-10)
    # exactly component-block preconditioned: 1 +- sqrt(ab / ((1+a)(1+b)))
    _, B1, B2 = _comp_block_precond(A, n0)
    MA = np.concatenate([B1 @ A[:n0], B2 @ A[n0:]])
    evm = np.sort(np.linalg.eigvals(MA).real)
    s = np.sqrt(aa * bb / ((1 + aa) * (1 + bb))).ravel()
    refm = np.sort(np.concatenate([1 - s, 1 + s]))
    np.testing.assert_allclose(evm, refm, rtol=1e-9, atol=1e-9)
    kappa, kappa_m = ev[-1] / ev[0], evm[-1] / evm[0]
    assert abs(kappa - (1 + 2 * c / dx ** 2)) <= 1e-9 * kappa
    assert abs(kappa_m - kappa) <= 1e-6 * kappa


def test_position_block_inverse_on_truncated_local_system():
    """A sweep's local system below full rank (decaying jet, 64 x 64, chi =
    16, centre at site 2, the stage step that gives the benchmark's
    mu h^2 / dx^2 of about 290): the exact inverse of the 4 x 4 position
    blocks over omega -- the block form the learned network predicts, at its
    best -- does not lower the warm-started CG iteration count (71 against
    65).  The exact inverse of the two component blocks does here (31), but
    it is a dense factorisation of a (4 chi^2)-square matrix per component
    and local solve: at chi = 128, 65536^3 / 3 = 9e13 flops against 1.2e9
    per CG iteration."""
    n, chi = 6, 16
    dx = 1.0 / (1 << n)
    h = (290.0 * dx * dx / 2.5e5) ** 0.5
    u = I.decaying_jet(n)
    b = [M.tt_svd(u[i], chi, 1e-12)[0] for i in range(2)]
    a = [M.scale(x, 0.25) for x in b]
    prm = S.Params(re=1e7, dt=3 * h, chi=chi, dx=dx)
    A, rhs, x0, n0, shape = _local_matrix(a, b, h, prm, 2)
    plain = _pcg_iters(A, rhs, x0, lambda r: r)
    comp, _, _ = _comp_block_precond(A, n0)
    with_comp = _pcg_iters(A, rhs, x0, comp)
    # 4 x 4 blocks over omega at every (component, alpha, beta) position
    P = np.zeros_like(A)
    for i in range(2):
        l, _, r = shape[i]
        for al in range(l):
            for be in range(r):
                idx = [i * n0 + (al * 4 + w) * r + be for w in range(4)]
                P[np.ix_(idx, idx)] = np.linalg.inv(A[np.ix_(idx, idx)])
    with_pos = _pcg_iters(A, rhs, x0, lambda v: P @ v)
    assert plain > 50
    assert with_pos >= plain, (plain, with_pos)
    assert with_comp < plain, (plain, with_comp)


def _kron_sum_fit(K, l, r):
    """Frobenius-nearest A (x) I (x) I + I (x) B (x) I + I (x) I (x) C to K
    (l*4*r square, index order (alpha, omega, beta)): the traceless parts of
    the scaled partial traces, the identity part carried by A."""
    K6 = K.reshape(l, 4, r, l, 4, r)
    T = np.trace(K)
    A = np.einsum('awbcwb->ac', K6) / (4 * r)
    B = np.einsum('awbavb->wv', K6) / (l * r) - T / (4 * l * r) * np.eye(4)
    C = np.einsum('awbawc->bc', K6) / (4 * l) - T / (4 * l * r) * np.eye(r)
    return A, B, C


def _kron_sum_inverse(A, B, C, l, r):
    la, Qa = np.linalg.eigh(0.5 * (A + A.T))
    lb, Qb = np.linalg.eigh(0.5 * (B + B.T))
    lc, Qc = np.linalg.eigh(0.5 * (C + C.T))
    lam = np.maximum(1.0 + la[:, None, None] + lb[None, :, None] + lc[None, None, :], 1.0)

    def apply(x):
        Y = np.einsum('ia,iwb,wv,bc->avc', Qa, x.reshape(l, 4, r), Qb, Qc, optimize=True) / lam
        return np.einsum('ai,avc,wv,bc->iwb', Qa, Y, Qb, Qc, optimize=True).ravel()
    return apply


def _kron_prod_fit(K, l, r, iters=30):
    """Frobenius-nearest X (x) Y (x) Z to K by alternating least squares."""
    K6 = K.reshape(l, 4, r, l, 4, r)
    X, Y, Z = np.eye(l), np.eye(4), np.eye(r)
    for _ in range(iters):
        X = np.einsum('awbcvd,wv,bd->ac', K6, Y, Z, optimize=True) / (np.sum(Y * Y) * np.sum(Z * Z))
        Y = np.einsum('awbcvd,ac,bd->wv', K6, X, Z, optimize=True) / (np.sum(X * X) * np.sum(Z * Z))
        Z = np.einsum('awbcvd,ac,wv->bd', K6, X, Y, optimize=True) / (np.sum(X * X) * np.sum(Y * Y))
    Xi, Yi, Zi = np.linalg.inv(X), np.linalg.inv(Y), np.linalg.inv(Z)
    return lambda x: np.einsum('ac,wv,bd,cvd->awb', Xi, Yi, Zi, x.reshape(l, 4, r),
                               optimize=True).ravel()


def test_kronecker_component_preconditioners_do_not_pay_over_a_sweep():
    """Decaying jet, 64 x 64, chi = 16, mu h^2 / dx^2 = 290 (the benchmark's
    stage ratio): the warm-started CG iterations of the local solves at
    sites 1..4 sum to more with either Kronecker form than without a
    preconditioner, although each approximates its block to about 30%."""
    n, chi = 6, 16
    dx = 1.0 / (1 << n)
    h = (290.0 * dx * dx / 2.5e5) ** 0.5
    u = I.decaying_jet(n)
    b = [M.tt_svd(u[i], chi, 1e-12)[0] for i in range(2)]
    a = [M.scale(x, 0.25) for x in b]
    prm = S.Params(re=1e7, dt=3 * h, chi=chi, dx=dx)
    plain = ksum = kprod = 0
    for d in range(1, 5):
        A, rhs, x0, n0, shape = _local_matrix(a, b, h, prm, d)
        N = A.shape[0]
        sums, prods = [], []
        for i in range(2):
            l, _, r = shape[i]
            sl = slice(0, n0) if i == 0 else slice(n0, N)
            Aii = A[sl, sl]
            K = Aii - np.eye(Aii.shape[0])
            Af, Bf, Cf = _kron_sum_fit(K, l, r)
            fit = (np.kron(np.kron(Af, np.eye(4)), np.eye(r))
                   + np.kron(np.kron(np.eye(l), Bf), np.eye(r)) + np.kron(np.eye(4 * l), Cf))
            assert np.linalg.norm(K - fit) <= 0.5 * np.linalg.norm(K)
            sums.append(_kron_sum_inverse(Af, Bf, Cf, l, r))
            prods.append(_kron_prod_fit(Aii, l, r))
        plain += _pcg_iters(A, rhs, x0, lambda v: v)
        ksum += _pcg_iters(A, rhs, x0, lambda v: np.concatenate([sums[0](v[:n0]), sums[1](v[n0:])]))
        kprod += _pcg_iters(A, rhs, x0,
                            lambda v: np.concatenate([prods[0](v[:n0]), prods[1](v[n0:])]))
    assert ksum > plain and kprod > plain, (plain, ksum, kprod)
