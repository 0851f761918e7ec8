"""Pins of the Schmidt-count oracle (bond dimension chi_l(eps) of a dense
field, the paper's MPS compression-efficiency analysis, Eq. epsilon):
closed-form quantics ranks of simple fields, a prescribed spectrum at one
bipartition, and the tail rule at its boundary."""
import numpy as np
import pytest

from oracle import mps as M
from oracle import schmidt as Sc


def _grid(n):
    N = 1 << n
    x = np.arange(N) / N
    return np.meshgrid(x, x, indexing='ij')


def test_closed_form_ranks():
    n = 5
    X, Y = _grid(n)
    # constant: rank 1; sin(2 pi x): the coarsest bit only flips the sign
    # (rank 1 at the first cut), deeper cuts split sin(a + b) into two terms
    assert Sc.schmidt_counts(np.ones_like(X), 1e-12) == [1] * (n - 1)
    assert Sc.schmidt_counts(np.sin(2 * np.pi * X), 1e-12) == [1, 2, 2, 2]
    # a product of an x-field and a y-field: ranks multiply
    assert Sc.schmidt_counts(np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y), 1e-12) == [1, 4, 4, 4]
    # exp(2 pi i (x + y)) has rank 1, so sin(2 pi (x + y)) has rank 2
    assert Sc.schmidt_counts(np.sin(2 * np.pi * (X + Y)), 1e-12) == [1, 2, 2, 2]


@pytest.mark.parametrize('l', [1, 2, 3])
def test_prescribed_spectrum_at_one_bipartition(l):
    n = 4
    rng = np.random.default_rng(l)
    r = min(4 ** l, 4 ** (n - l))
    s = np.sort(rng.uniform(0.0, 1.0, r) ** 6)[::-1]
    Q1, _ = np.linalg.qr(rng.standard_normal((4 ** l, r)))
    Q2, _ = np.linalg.qr(rng.standard_normal((4 ** (n - l), r)))
    A = (Q1 * s) @ Q2.T
    U = M.decode(A.reshape(-1), n)
    got = Sc.schmidt_values(U)[l - 1]
    np.testing.assert_allclose(got, s, atol=1e-13)
    for eps in (1e-1, 1e-2, 1e-3):
        assert Sc.schmidt_counts(U, eps)[l - 1] == Sc.count_for_eps(s, eps)


def test_tail_rule():
    assert Sc.count_for_eps([4.0, 3.0], 0.6) == 1        # tail 9 <= 0.36 * 25
    assert Sc.count_for_eps([4.0, 3.0], 0.59) == 2
    assert Sc.count_for_eps([4.0, 3.0, 0.0], 0.0) == 2    # exact rank
    assert Sc.count_for_eps([4.0, 3.0], 1.0) == 1         # at least one value
    assert Sc.count_for_eps([0.0, 0.0], 0.1) == 0         # zero field
