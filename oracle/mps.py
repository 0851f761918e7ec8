"""Quantics MPS algebra in float64 -- test oracle (see package docstring).

Conventions (paper Sec. II.B "Algorithmic Building Blocks"):
  * grid N = 2**n per side, values U[x1, x2];
  * site k (0-based, site 0 = coarsest scale) carries the physical index
    omega_k = 2*bit_k(x1) + bit_k(x2), bit 0 being the most significant bit;
  * an MPS is a list of float64 cores of shape (l_k, 4, r_k) with l_0 = r_{n-1} = 1;
  * the dense vector of an MPS is ordered with site 0 most significant
    (Morton / Z order of the grid).
"""
import numpy as np


# --------------------------------------------------------------------------
# encoding (Sec. II.B, quantics interleaving of the two coordinates' bits)
# --------------------------------------------------------------------------
def morton_index(n):
    """idx[x1, x2] = position of grid point (x1, x2) in the quantics vector."""
    N = 1 << n
    x1 = np.arange(N)[:, None]
    x2 = np.arange(N)[None, :]
    idx = np.zeros((N, N), dtype=np.int64)
    for k in range(n):
        b1 = (x1 >> (n - 1 - k)) & 1
        b2 = (x2 >> (n - 1 - k)) & 1
        idx += (2 * b1 + b2) << (2 * (n - 1 - k))
    return idx


def encode(U):
    """Dense N x N grid -> quantics vector of length 4**n."""
    N = U.shape[0]
    n = N.bit_length() - 1
    T = np.empty(N * N, dtype=U.dtype)
    T[morton_index(n)] = U
    return T


def decode(T, n):
    """Quantics vector -> dense N x N grid."""
    return T[morton_index(n)]


# --------------------------------------------------------------------------
# basic MPS helpers
# --------------------------------------------------------------------------
def bonds(cores):
    """Bond list [1, r_0, r_1, ..., r_{n-2}, 1] (length n + 1)."""
    return [cores[0].shape[0]] + [c.shape[2] for c in cores]


def structural_bound(n, k):
    """Largest useful bond dimension between sites k-1 and k: min(4**k, 4**(n-k))."""
    return min(4 ** k, 4 ** (n - k))


def to_vector(cores):
    """Contract all cores into the 4**n quantics vector."""
    v = cores[0].reshape(4, -1)
    for c in cores[1:]:
        v = (v @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    return v.reshape(-1)


def to_dense(cores):
    n = len(cores)
    return decode(to_vector(cores), n)


def values_at(cores, pts):
    """Field values at grid points pts[p] = (x1, x2): the product over sites
    of the core matrices C_k[:, omega_k, :] with omega_k = 2 bit_k(x1) +
    bit_k(x2), bit 0 the most significant (the encoding of Sec. II.B)."""
    n = len(cores)
    pts = np.asarray(pts)
    out = np.empty(len(pts))
    for p, (x1, x2) in enumerate(pts):
        row = np.ones((1, 1))
        for k in range(n):
            w = 2 * ((int(x1) >> (n - 1 - k)) & 1) + ((int(x2) >> (n - 1 - k)) & 1)
            row = row @ cores[k][:, w, :]
        out[p] = row[0, 0]
    return out


def copy(cores):
    return [c.copy() for c in cores]


def scale(cores, s):
    """s * x, folding the scalar into site 0."""
    out = copy(cores)
    out[0] = out[0] * s
    return out


def inner(x, y):
    """<x|y> by a left-to-right transfer-matrix contraction."""
    E = np.ones((1, 1))
    for a, b in zip(x, y):
        E = np.einsum('ab,awc,bwd->cd', E, a, b)
    return float(E[0, 0])


def norm_sq(x):
    return inner(x, x)


# --------------------------------------------------------------------------
# factorisations with a fixed sign convention
# --------------------------------------------------------------------------
def qr_pos(M):
    """Reduced QR with a non-negative diagonal of R (sign fixed so that two
    correct implementations produce the same factors for full-rank M)."""
    Q, R = np.linalg.qr(M, mode='reduced')
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def shift_right(cores, d):
    """Move the orthogonality centre from site d to d+1 (QR of site d)."""
    l, _, r = cores[d].shape
    Q, R = qr_pos(cores[d].reshape(l * 4, r))
    cores[d] = Q.reshape(l, 4, Q.shape[1])
    cores[d + 1] = np.einsum('ab,bwc->awc', R, cores[d + 1])


def shift_left(cores, d):
    """Move the orthogonality centre from site d to d-1 (LQ of site d)."""
    l, _, r = cores[d].shape
    Q, R = qr_pos(cores[d].reshape(l, 4 * r).T)
    cores[d] = Q.T.reshape(Q.shape[1], 4, r)
    cores[d - 1] = np.einsum('awb,bc->awc', cores[d - 1], R.T)


def right_canonicalize(cores):
    """Right-orthogonalise sites n-1..1; the centre ends at site 0."""
    out = copy(cores)
    for d in range(len(out) - 1, 0, -1):
        shift_left(out, d)
    return out


def left_canonicalize(cores):
    out = copy(cores)
    for d in range(len(out) - 1):
        shift_right(out, d)
    return out


def _keep(S, chi, cap, rtol):
    """Number of singular values kept: min(chi, structural cap, #sigma > rtol*sigma_max)."""
    if S.size == 0 or S[0] == 0.0:
        return 1
    k = min(chi, cap, S.size)
    if rtol > 0.0:
        k = min(k, int(np.count_nonzero(S > rtol * S[0])))
    return max(k, 1)


# --------------------------------------------------------------------------
# dense -> MPS (TT-SVD), the input compression of the initial velocities
# --------------------------------------------------------------------------
def tt_svd(U, chi, rtol=0.0):
    """Sequential truncated SVDs of the unfoldings (input preparation).

    Returns (cores, discarded_sq).
    """
    N = U.shape[0]
    n = N.bit_length() - 1
    M = encode(np.asarray(U, dtype=np.float64)).reshape(4, -1)
    cores, l, disc = [], 1, 0.0
    for k in range(n - 1):
        M = M.reshape(l * 4, -1)
        Uu, S, Vt = np.linalg.svd(M, full_matrices=False)
        r = _keep(S, chi, structural_bound(n, k + 1), rtol)
        disc += float(np.sum(S[r:] ** 2))
        cores.append(Uu[:, :r].reshape(l, 4, r))
        M = S[:r, None] * Vt[:r]
        l = r
    cores.append(M.reshape(l, 4, 1))
    return cores, disc


# --------------------------------------------------------------------------
# exact MPS algebra
# --------------------------------------------------------------------------
def add(coefs, xs):
    """y = sum_k c_k x_k; bonds add, cores block-diagonal, coefficients folded
    into site 0 (paper Sec. II.C: the RK4 step is a sum of four Euler steps)."""
    n = len(xs[0])
    if n == 1:
        return [sum(c * x[0] for c, x in zip(coefs, xs))]
    out = []
    for s in range(n):
        ls = [x[s].shape[0] for x in xs]
        rs = [x[s].shape[2] for x in xs]
        if s == 0:
            core = np.zeros((1, 4, sum(rs)))
            o = 0
            for c, x in zip(coefs, xs):
                core[:, :, o:o + x[0].shape[2]] = c * x[0]
                o += x[0].shape[2]
        elif s == n - 1:
            core = np.zeros((sum(ls), 4, 1))
            o = 0
            for x in xs:
                core[o:o + x[s].shape[0]] = x[s]
                o += x[s].shape[0]
        else:
            core = np.zeros((sum(ls), 4, sum(rs)))
            ol = orr = 0
            for x in xs:
                a, _, b = x[s].shape
                core[ol:ol + a, :, orr:orr + b] = x[s]
                ol += a
                orr += b
        out.append(core)
    return out


def hadamard(a, b):
    """Pointwise product a*b: y[(al,al'), w, (be,be')] = A[al,w,be] B[al',w,be']
    (paper Sec. II.B, copy tensors delta_{www}); bond = chi_a * chi_b."""
    out = []
    for A, B in zip(a, b):
        la, _, ra = A.shape
        lb, _, rb = B.shape
        out.append(np.einsum('awb,cwd->acwbd', A, B).reshape(la * lb, 4, ra * rb))
    return out


def apply_mpo(W, x):
    """y = W x: y[(a,al), w, (b,be)] = sum_w' W[a,w,w',b] x[al,w',be]
    (the MPO's first physical index is the output, the second contracts with
    the MPS, App. A)."""
    out = []
    for Wc, X in zip(W, x):
        wl, _, _, wr = Wc.shape
        l, _, r = X.shape
        out.append(np.einsum('awvb,cvd->acwbd', Wc, X).reshape(wl * l, 4, wr * r))
    return out


def truncate(y, chi, rtol=0.0):
    """TT-rounding: left-to-right QR sweep, then right-to-left SVD keeping
    min(chi, structural bound, #sigma > rtol*sigma_max) values per bond
    (paper Sec. II.C: compression back to bond dimension chi by repeated
    SVDs).  The centre ends at site 0.  Returns (cores, discarded_sq)."""
    n = len(y)
    x = left_canonicalize(y)
    disc = 0.0
    for k in range(n - 1, 0, -1):
        l, _, r = x[k].shape
        Uu, S, Vt = np.linalg.svd(x[k].reshape(l, 4 * r), full_matrices=False)
        keep = _keep(S, chi, structural_bound(n, k), rtol)
        disc += float(np.sum(S[keep:] ** 2))
        x[k] = Vt[:keep].reshape(keep, 4, r)
        x[k - 1] = np.einsum('awb,bc->awc', x[k - 1], Uu[:, :keep] * S[None, :keep])
    return x, disc


def rel_l2(x, y):
    """||x - y|| / ||y|| computed through the MPS difference (no cancellation
    of large inner products)."""
    d = right_canonicalize(add([1.0, -1.0], [x, y]))
    return float(np.linalg.norm(d[0])) / float(np.linalg.norm(right_canonicalize(y)[0]))
