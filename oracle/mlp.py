"""Float64 reference of the learned block preconditioner's network -- test oracle.

Test infrastructure only: nothing in the library imports this module.

The preconditioner of the local CG solves (an addition; the paper's local
systems, App. B Eq. big_LS, are solved by plain CG) is a 3-layer perceptron
applied independently to every (alpha, beta) position of a centre tensor:

    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,

x = 16 features of the 4 x 4 diagonal block of the local matrix at that
position, y = the 10 entries of a lower-triangular factor L (row-major lower
triangle, diagonal through exp); the block of the preconditioner is
M = L L^T (symmetric positive definite by construction).  Training minimises
||z - M A z||^2 / ||z||^2 over random probes z.

`round_op` optionally rounds every matrix-product operand before the product,
to reproduce a kernel whose products take rounded operands (bfloat16 in the
library: float64 -> float32 -> bfloat16, round to nearest even at each step);
the sums themselves stay float64 here.

Pins (tests/test_oracle_mlp.py): backward pass against central finite
differences of the forward pass; factor gradient against finite differences;
M is SPD; the bfloat16 rounding against exhaustive properties of the format.
"""
import numpy as np

TRI = [(r, c) for r in range(4) for c in range(r + 1)]   # 10 lower-triangle entries
N_IN, WIDTH, N_OUT = 16, 256, 10


def bf16(x):
    """Round float64 values to bfloat16 via float32, round to nearest even at
    both steps (returned as float64)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return b.view(np.float32).astype(np.float64)


def _id(x):
    return x


def init(n_in=N_IN, width=WIDTH, n_out=N_OUT, seed=0):
    rng = np.random.default_rng(seed)
    return {
        'W1': rng.standard_normal((width, n_in)) * np.sqrt(2.0 / n_in),
        'b1': np.zeros(width),
        'W2': rng.standard_normal((width, width)) * np.sqrt(2.0 / width),
        'b2': np.zeros(width),
        'W3': rng.standard_normal((n_out, width)) * (0.01 / np.sqrt(width)),
        'b3': np.zeros(n_out),
    }


ORDER = ('W1', 'b1', 'W2', 'b2', 'W3', 'b3')


def flatten(p):
    return np.concatenate([p[k].ravel() for k in ORDER])


def unflatten(w, n_in=N_IN, width=WIDTH, n_out=N_OUT):
    shapes = {'W1': (width, n_in), 'b1': (width,), 'W2': (width, width), 'b2': (width,),
              'W3': (n_out, width), 'b3': (n_out,)}
    p, o = {}, 0
    for k in ORDER:
        n = int(np.prod(shapes[k]))
        p[k] = np.array(w[o:o + n]).reshape(shapes[k])
        o += n
    assert o == len(w)
    return p


def forward(p, X, round_op=_id):
    """X: (batch, n_in) -> (y, cache)."""
    R = round_op
    z1 = R(X) @ R(p['W1']).T + p['b1']
    h1 = np.maximum(z1, 0.0)
    z2 = R(h1) @ R(p['W2']).T + p['b2']
    h2 = np.maximum(z2, 0.0)
    y = R(h2) @ R(p['W3']).T + p['b3']
    return y, (X, z1, h1, z2, h2)


def backward(p, cache, dy, round_op=_id):
    """Gradients of sum(dy * y) with respect to the parameters."""
    R = round_op
    X, z1, h1, z2, h2 = cache
    g = {'W3': R(dy).T @ R(h2), 'b3': dy.sum(0)}
    dh2 = R(dy) @ R(p['W3'])
    dz2 = dh2 * (z2 > 0)
    g['W2'] = R(dz2).T @ R(h1)
    g['b2'] = dz2.sum(0)
    dh1 = R(dz2) @ R(p['W2'])
    dz1 = dh1 * (z1 > 0)
    g['W1'] = R(dz1).T @ R(X)
    g['b1'] = dz1.sum(0)
    return g


def factor(y):
    """(batch, 10) -> lower-triangular (batch, 4, 4) with exp on the diagonal."""
    L = np.zeros((y.shape[0], 4, 4))
    for t, (r, c) in enumerate(TRI):
        L[:, r, c] = np.exp(y[:, t]) if r == c else y[:, t]
    return L


def factor_grad(y, dL):
    """Gradient with respect to y of sum(dL * factor(y))."""
    dy = np.zeros_like(y)
    for t, (r, c) in enumerate(TRI):
        dy[:, t] = dL[:, r, c] * (np.exp(y[:, t]) if r == c else 1.0)
    return dy


def probe_loss(y, z, az):
    """Loss sum_p |z_p - M_p az_p|^2 / sum_p |z_p|^2 with M_p = L_p L_p^T,
    L = factor(y); z, az: (batch, 4).  Returns (loss, dloss/dy)."""
    L = factor(y)
    M = L @ L.transpose(0, 2, 1)
    res = z - np.einsum('pij,pj->pi', M, az)
    zz = float(np.sum(z * z))
    loss = float(np.sum(res * res)) / zz
    G = -2.0 / zz * np.einsum('pi,pj->pij', res, az)        # dloss/dM
    dL = (G + G.transpose(0, 2, 1)) @ L                      # through M = L L^T
    return loss, factor_grad(y, dL)
