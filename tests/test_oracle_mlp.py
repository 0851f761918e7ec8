"""Pins of the preconditioner network's float64 oracle: gradients equal
central finite differences of the forward pass, the factor yields SPD blocks,
and the bfloat16 rounding follows the format's definition."""
import numpy as np

from oracle import mlp


def _fd_check(f, x, g, rng, eps=1e-6, count=12, tol=1e-6):
    flat = x.reshape(-1)
    gf = g.reshape(-1)
    for idx in rng.choice(flat.size, size=min(count, flat.size), replace=False):
        old = flat[idx]
        flat[idx] = old + eps
        fp = f()
        flat[idx] = old - eps
        fm = f()
        flat[idx] = old
        num = (fp - fm) / (2 * eps)
        assert abs(num - gf[idx]) <= tol * (1 + abs(num)), (idx, num, gf[idx])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init(12, width=16, n_out=10, seed=2)
    p['W3'] = rng.standard_normal(p['W3'].shape) * 0.3
    X = rng.standard_normal((5, 12))
    dy = rng.standard_normal((5, 10))
    y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, dy)
    for name in mlp.ORDER:
        _fd_check(lambda: float(np.sum(dy * mlp.forward(p, X)[0])), p[name], g[name], rng)


def test_factor_gives_spd_blocks_and_gradient():
    rng = np.random.default_rng(3)
    y = rng.standard_normal((4, 10))
    L = mlp.factor(y)
    assert np.all(np.triu(L, 1) == 0)
    M = L @ L.transpose(0, 2, 1)
    assert np.all(np.linalg.eigvalsh(M) > 0)
    dL = rng.standard_normal((4, 4, 4))
    dy = mlp.factor_grad(y, dL)
    _fd_check(lambda: float(np.sum(dL * mlp.factor(y))), y, dy, rng, count=40)


def test_probe_loss_gradient_and_exact_inverse():
    rng = np.random.default_rng(4)
    y = rng.standard_normal((6, 10)) * 0.5
    z = rng.standard_normal((6, 4))
    az = rng.standard_normal((6, 4))
    loss, dy = mlp.probe_loss(y, z, az)
    _fd_check(lambda: mlp.probe_loss(y, z, az)[0], y, dy, rng, count=40)
    # with A block-diagonal SPD and M = A^-1 (Cholesky factor of the inverse)
    # the loss vanishes for every probe
    B = rng.standard_normal((6, 4, 4))
    A = B @ B.transpose(0, 2, 1) + 4 * np.eye(4)
    C = np.linalg.cholesky(np.linalg.inv(A))
    ye = np.zeros((6, 10))
    for t, (r, c) in enumerate(mlp.TRI):
        ye[:, t] = np.log(C[:, r, c]) if r == c else C[:, r, c]
    l0, _ = mlp.probe_loss(ye, z, np.einsum('pij,pj->pi', A, z))
    assert l0 < 1e-24


def test_bf16_rounding():
    # exactly representable values are kept
    vals = np.array([0.0, 1.0, -2.0, 0.5, 1.0 + 2.0 ** -7, 3.0 * 2.0 ** -20, 65280.0])
    assert np.array_equal(mlp.bf16(vals), vals)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert mlp.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    # relative error at most 2^-8 (half an ulp of an 8-bit significand) plus
    # 2^-24 from the float32 step, and
    # every result carries at most 8 significant bits
    x = np.random.default_rng(5).standard_normal(10000) * 10.0 ** np.random.default_rng(6).uniform(-5, 5, 10000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= (2.0 ** -8 + 2.0 ** -24) * np.abs(x))
    m, _ = np.frexp(r)
    assert np.all(m * 2 ** 8 == np.round(m * 2 ** 8))


def test_flatten_layout():
    p = mlp.init(seed=7)
    w = mlp.flatten(p)
    assert w.size == 16 * 256 + 256 + 256 * 256 + 256 + 10 * 256 + 10
    q = mlp.unflatten(w)
    for k in mlp.ORDER:
        assert np.array_equal(p[k], q[k])
