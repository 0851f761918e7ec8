"""Schmidt spectra and the bond dimension chi_l(eps) of a dense field -- test
oracle (see package docstring).

The analysis of the paper's section on MPS compression efficiency: the
field on the N x N grid (N = 2^n) is the quantics state of n sites; the
bipartition l (sites 0..l-1 against l..n-1) has the Schmidt values of the
4^l x 4^(n-l) unfolding of the site-ordered vector, and chi_l(eps) is the
least number of them whose discarded tail keeps the relative L2 error of
that bipartition within eps (Eq. epsilon), chi = max_l chi_l.  Written as
the definition: one dense SVD per bipartition.
"""
import numpy as np

from . import mps as M


def schmidt_values(U):
    """Singular values (descending) of every bipartition l = 1 .. n-1."""
    N = U.shape[0]
    n = N.bit_length() - 1
    T = M.encode(np.asarray(U, dtype=np.float64))
    return [np.linalg.svd(T.reshape(4 ** l, -1), compute_uv=False) for l in range(1, n)]


def count_for_eps(s, eps):
    """Least chi with sqrt(sum_{k >= chi} s_k^2) <= eps sqrt(sum_k s_k^2)
    (s descending); at least 1 for a nonzero field, 0 for a zero one."""
    s2 = np.asarray(s, dtype=np.float64) ** 2
    total = float(np.sum(s2))
    if total == 0.0:
        return 0
    # tail[c] = sum_{k >= c} s_k^2 for c = 0 .. len(s)
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])
    ok = np.nonzero(tail <= eps * eps * total)[0]
    return max(1, int(ok[0]))


def schmidt_counts(U, eps):
    """chi_l(eps) for every bipartition l = 1 .. n-1."""
    return [count_for_eps(s, eps) for s in schmidt_values(U)]
