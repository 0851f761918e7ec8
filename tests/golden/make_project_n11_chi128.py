"""Writes project_n11_chi128.txt: the float64 oracle's one-sweep projection
(App. B, Eq. Theta; the one-site sweep of Sec. II.C) at 2048 x 2048 (11
sites) with every bond at its structural bound min(128, 4^k, 4^(11-k)),
sampled at seeded grid points.

The input is seeded random cores (b, normalised to unit norm), a = b / 4,
h = dt / 6 with dt = 5e-5, Re = 1e7, guess a, one sweep, CG relative
tolerance 1e-12.  Only the oracle and the seeded input generators run here;
about three minutes on eight host threads.

    python tests/golden/make_project_n11_chi128.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import mps as M  # noqa: E402
from oracle import sweep as S  # noqa: E402
from paper_2406_17823_amd import inputs as I  # noqa: E402

N_SITES, CHI, SEED, DT, RE = 11, 128, 1100, 5e-5, 1e7
N_POINTS, POINT_SEED = 1024, 1101
OUT = os.path.join(HERE, 'project_n11_chi128.txt')


def case():
    """The seeded input: (a, b, h, Params) of the projection."""
    bonds = I.canonical_bonds(N_SITES, CHI)
    b = []
    for i in range(2):
        x = I.random_cores(bonds, SEED + i)
        b.append(M.scale(x, 1.0 / np.sqrt(M.norm_sq(x))))
    a = [M.scale(x, 0.25) for x in b]
    prm = S.Params(re=RE, dt=DT, chi=CHI, dx=1.0 / (1 << N_SITES), max_sweeps=1, cg_rtol=1e-12)
    return a, b, DT / 6, prm


def points():
    rng = np.random.default_rng(POINT_SEED)
    N = 1 << N_SITES
    return rng.integers(0, N, size=(N_POINTS, 2))


def main():
    a, b, h, prm = case()
    st = S.Stats()
    t0 = time.perf_counter()
    v = S.project(a, b, h, prm, a, st)
    el = time.perf_counter() - t0
    pts = points()
    vals = [M.values_at(v[i], pts) for i in range(2)]
    with open(OUT, 'w') as f:
        f.write('# float64 oracle, one-sweep projection at 2048 x 2048, chi = 128, saturated bonds\n')
        f.write('# written by tests/golden/make_project_n11_chi128.py (oracle only)\n')
        f.write(f'# oracle: {el:.0f} s, {st.cg_solves} CG solves, {st.cg_iters_total} CG iterations\n')
        f.write(f'n {N_SITES}\nchi {CHI}\nseed {SEED}\npoint_seed {POINT_SEED}\n')
        for i in range(2):
            f.write(f'bonds{i} ' + ' '.join(str(x) for x in M.bonds(v[i])) + '\n')
            f.write(f'normsq{i} {M.norm_sq(v[i]):.17e}\n')
        f.write(f'points {N_POINTS}\n')
        for p, (x1, x2) in enumerate(pts):
            f.write(f'{x1} {x2} {vals[0][p]:.17e} {vals[1][p]:.17e}\n')
    print('wrote', OUT, f'{el:.0f} s', st)


if __name__ == '__main__':
    main()
