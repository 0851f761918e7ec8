"""Finite-difference MPOs -- test oracle (see package docstring).

Paper Sec. II.B (Eq. fdm, the central-difference operator D_1) and App. A
(carry table of the central node C, boundary vectors L and R).

An MPO is a list of float64 cores W[a, w, w', b]: a is the bond towards the
coarser (more significant) site, b towards the finer site, w is the output
physical index and w' the one contracted with the MPS.  The boundary vectors
are folded into the first and last cores, so core 0 has a = 1 and the last
core has b = 1.
"""
import numpy as np

# operations requested by the finer sites through the bond alpha_{m+1}:
# 0 = leave the bit, 1 = add one, 2 = subtract one (App. A)
_DELTA = {0: 0, 1: +1, 2: -1}


def carry_core(axis):
    """Central node C[alpha_m, omega, omega', alpha_{m+1}] of App. A.

    axis 1 acts on the x1 bit (the high bit of omega), axis 2 on the x2 bit.
    For an incoming request op = alpha_{m+1} the output point with bit b reads
    the input point whose bit is b + delta(op); when that leaves {0, 1} the
    bit wraps and the request is passed on to the coarser site (alpha_m = op),
    otherwise alpha_m = 0.
    """
    shift = 1 if axis == 1 else 0
    C = np.zeros((3, 4, 4, 3))
    for op in range(3):
        for w in range(4):
            bit = (w >> shift) & 1
            nb = bit + _DELTA[op]
            carry = 0 if 0 <= nb <= 1 else op
            w_in = (w & ~(1 << shift)) | ((nb % 2) << shift)
            C[carry, w, w_in, op] = 1.0
    return C


def boundary_vectors(order, dx):
    """L = (1, 1, 1) (periodic wrap: any carry out of the coarsest bit is
    dropped); R picks the stencil weights of the identity / +1 / -1 shifts.

    order 1: R = (0, 1, -1) / (2 dx)        (App. A)
    order 2: R = (-2, 1, 1) / dx**2         (three-point second difference,
                                              same carry logic, Sec. II.B)
    """
    L = np.ones(3)
    if order == 1:
        R = np.array([0.0, 1.0, -1.0]) / (2.0 * dx)
    elif order == 2:
        R = np.array([-2.0, 1.0, 1.0]) / (dx * dx)
    else:
        raise ValueError("order must be 1 or 2")
    return L, R


def mpo_from_core(n, C, L, R):
    if n == 1:
        return [np.einsum('a,awvb,b->wv', L, C, R).reshape(1, 4, 4, 1)]
    first = np.einsum('a,awvb->wvb', L, C)[None]
    last = np.einsum('awvb,b->awv', C, R)[..., None]
    return [first] + [C.copy() for _ in range(n - 2)] + [last]


def derivative_mpo(n, axis, order, dx):
    """D_axis (order 1, central difference) or the three-point D_axis^2."""
    L, R = boundary_vectors(order, dx)
    return mpo_from_core(n, carry_core(axis), L, R)


def mpo_sum(W1, W2):
    """W1 + W2 as one MPO (bonds add)."""
    n = len(W1)
    if n == 1:
        return [W1[0] + W2[0]]
    out = []
    for s, (A, B) in enumerate(zip(W1, W2)):
        a1, _, _, b1 = A.shape
        a2, _, _, b2 = B.shape
        if s == 0:
            out.append(np.concatenate([A, B], axis=3))
        elif s == n - 1:
            out.append(np.concatenate([A, B], axis=0))
        else:
            c = np.zeros((a1 + a2, 4, 4, b1 + b2))
            c[:a1, :, :, :b1] = A
            c[a1:, :, :, b1:] = B
            out.append(c)
    return out


def mpo_compose(W1, W2):
    """The operator W1 W2 (W2 acts first)."""
    out = []
    for A, B in zip(W1, W2):
        a1, _, _, b1 = A.shape
        a2, _, _, b2 = B.shape
        out.append(np.einsum('awub,cuvd->acwvbd', A, B).reshape(a1 * a2, 4, 4, b1 * b2))
    return out


def mpo_transpose(W):
    """Transpose of the operator: swap the two physical indices."""
    return [c.transpose(0, 2, 1, 3).copy() for c in W]


def laplacian_mpo(n, dx, lap_mode=0):
    """sum_j D_j^2 of the diffusion term (App. B, Eq. Theta).

    lap_mode 0: three-point second differences (bond 3 + 3);
    lap_mode 1: the literal D_j o D_j of the first-difference MPO (bond 9 + 9).
    """
    if lap_mode == 0:
        return mpo_sum(derivative_mpo(n, 1, 2, dx), derivative_mpo(n, 2, 2, dx))
    D1 = derivative_mpo(n, 1, 1, dx)
    D2 = derivative_mpo(n, 2, 1, dx)
    return mpo_sum(mpo_compose(D1, D1), mpo_compose(D2, D2))


def mpo_to_matrix(W):
    """Dense 4**n x 4**n matrix of an MPO (tiny n only); rows are outputs."""
    M = W[0].reshape(4, 4, -1)  # (w, w', b)
    for c in W[1:]:
        a, _, _, b = c.shape
        M = np.einsum('xya,awvb->xwyvb', M, c)
        M = M.reshape(M.shape[0] * 4, M.shape[2] * 4, b)
    return M[:, :, 0]
