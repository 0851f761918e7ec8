"""One-site variational sweep and the RK4 step -- test oracle.

App. B of the paper: each Euler step minimises
    Theta(v; a, b, h) = mu ||D_1 v_1 + D_2 v_2||^2
                        + || sum_i e_i [(v_i - a_i)/h + B_i(b)] ||^2
over MPS v_1, v_2.  With v_i in mixed-canonical form around site d
(Eq. mixed_canonical) and P_i the isometry that maps the centre tensor C_i to
the state, stationarity gives the coupled local system (Eqs. first/second,
big_LS)
    C_i + mu h^2 sum_j P_i^T D_i^T D_j P_j C_j = P_i^T a_i - h P_i^T B_i(b),
which is SPD and is solved by conjugate gradients (Sec. II.C).  Every term is
a tensor network whose left and right parts ("environments") are contracted
once and updated site by site (Sec. II.C, Fig. nonlinear_Ax(b)); the
convection term enters through MPOs built from b (copy tensors,
Sec. II.B), so the right-hand side is the exact projection of a - h B(b).
The sweep starts at the canonical centre, goes to the last site and back,
and stops when the relative change of sum_i <v_i|v_i> falls below a
tolerance (Sec. II.C) or after max_sweeps sweeps.

RK4 (App. B, Table RK4, Eqs. U1-U4): four minimisations with a = u/4,
h = dt/6, dt/3, dt/3, dt/6 and b = u, 3 U1 + u/4, 3/2 U2 + 5/8 u,
3 U3 + u/4; the new state is the sum U1 + U2 + U3 + U4 compressed to chi.

Explicit right-hand side (rhs_mode 1, the other reading of the Hadamard
term): B(b) is fitted once as a chi-bounded MPS w, a least-squares fit on
the bonds of b by the same one-site sweep with the B(b) networks alone (the
local matrix is the identity), and each minimisation then sees a - h w
through two layer-free networks per component.

RK1 and RK2 (App. B, Eqs. euler, midpoint_calc, full_calc): explicit Euler is
one minimisation with a = b = u, h = dt; the midpoint method takes
u_mid = argmin Theta(v; u, u, dt/2), then argmin Theta(v; u, u_mid, dt).
Every minimisation starts from the guess v = u (the paper does not say).
"""
from dataclasses import dataclass, replace

import numpy as np

from . import mps as M
from . import mpo as O


@dataclass
class Params:
    re: float
    dt: float
    chi: int
    dx: float
    mu: float = 2.5e5          # penalty factor (App. B)
    cg_rtol: float = 1e-12     # relative residual ||r|| / ||rhs||
    cg_maxit: int = 1000
    sweep_rtol: float = 0.0    # 0: always run max_sweeps sweeps
    max_sweeps: int = 2
    lap_mode: int = 0          # 0: three-point D_j^2, 1: D_j o D_j
    svd_rtol: float = 1e-12    # relative singular-value cutoff in truncation
    rhs_mode: int = 0          # 0: B(b) inside the networks, 1: B(b) fitted first
    fit_sweeps: int = 0        # sweeps of that fit (0: max_sweeps)


@dataclass
class Stats:
    sweeps: int = 0
    cg_iters_total: int = 0
    cg_iters_max: int = 0
    cg_solves: int = 0
    cg_maxit_hits: int = 0


def hadamard_mpo(b):
    """The MPO |b> (.) of Sec. II.B: each core of b contracted with delta_{www}."""
    return [np.einsum('awb,wv->awvb', c, np.eye(4)) for c in b]


_PATHS = {}


def _einsum(sub, *ops):
    """np.einsum with the pairwise contraction order looked up once per
    subscript/shape signature."""
    key = (sub,) + tuple(o.shape for o in ops)
    path = _PATHS.get(key)
    if path is None:
        path = np.einsum_path(sub, *ops, optimize=('greedy', 1 << 40))[0]
        _PATHS[key] = path
    return np.einsum(sub, *ops, optimize=path)


# --------------------------------------------------------------------------
# environments: E[alpha_bra, m_1, ..., m_p, alpha_ket], p = number of MPO layers
# --------------------------------------------------------------------------
def transfer_left(E, bra, layers, ket):
    if len(layers) == 0:
        return _einsum('ag,awb,gwc->bc', E, bra, ket)
    if len(layers) == 1:
        return _einsum('amg,awb,mwvn,gvc->bnc', E, bra, layers[0], ket)
    return _einsum('amog,awb,mwvn,ovup,guc->bnpc', E, bra, layers[0], layers[1], ket)


def transfer_right(E, bra, layers, ket):
    if len(layers) == 0:
        return _einsum('bc,awb,gwc->ag', E, bra, ket)
    if len(layers) == 1:
        return _einsum('bnc,awb,mwvn,gvc->amg', E, bra, layers[0], ket)
    return _einsum('bnpc,awb,mwvn,ovup,guc->amog', E, bra, layers[0], layers[1], ket)


def open_site(L, layers, ket, R):
    """The network with the bra tensor at the site removed: a tensor shaped
    like the centre, (alpha_{d-1}, omega_d, alpha_d)."""
    if len(layers) == 0:
        return _einsum('ag,gwc,bc->awb', L, ket, R)
    if len(layers) == 1:
        return _einsum('amg,mwvn,gvc,bnc->awb', L, layers[0], ket, R)
    return _einsum('amog,mwvn,ovup,guc,bnpc->awb', L, layers[0], layers[1], ket, R)


class Network:
    """<v_bra| W_1 ... W_p |ket> with ket a fixed MPS or one of the trial MPS."""

    def __init__(self, bra, layers, ket, coef):
        self.bra = bra          # component index of the bra
        self.layers = layers    # list of MPOs (lists of cores)
        self.ket = ket          # ('fixed', cores) or ('v', component)
        self.coef = coef
        self.L = None
        self.R = None

    def ket_core(self, v, d):
        return self.ket[1][d] if self.ket[0] == 'fixed' else v[self.ket[1]][d]

    def layer_cores(self, d):
        return [W[d] for W in self.layers]

    def trivial(self):
        return np.ones((1,) * (len(self.layers) + 2))

    def init(self, v, n):
        self.L = [None] * n
        self.R = [None] * n
        self.L[0] = self.trivial()
        self.R[n - 1] = self.trivial()
        for d in range(n - 1, 0, -1):
            self.R[d - 1] = transfer_right(self.R[d], v[self.bra][d], self.layer_cores(d),
                                           self.ket_core(v, d))

    def update_left(self, v, d):
        self.L[d + 1] = transfer_left(self.L[d], v[self.bra][d], self.layer_cores(d),
                                      self.ket_core(v, d))

    def update_right(self, v, d):
        self.R[d - 1] = transfer_right(self.R[d], v[self.bra][d], self.layer_cores(d),
                                       self.ket_core(v, d))

    def open(self, d, ket_core):
        return open_site(self.L[d], self.layer_cores(d), ket_core, self.R[d])


def build_networks(a, b, h, prm, n, w=None, fit=False):
    """Right-hand-side networks and penalty networks of the local system.

    fit: the networks of B_i(b) alone and no penalty (the local solution is
    the projected right-hand side: a least-squares fit of B(b) on the trial
    bonds); w given: the right-hand side a_i - h w_i from a fitted B."""
    D = [O.derivative_mpo(n, 1, 1, prm.dx), O.derivative_mpo(n, 2, 1, prm.dx)]
    DT = [O.mpo_transpose(W) for W in D]
    Lap = O.laplacian_mpo(n, prm.dx, prm.lap_mode)
    rhs = []
    if w is not None:
        for i in range(2):
            rhs.append(Network(i, [], ('fixed', a[i]), 1.0))
            rhs.append(Network(i, [], ('fixed', w[i]), -h))
    else:
        H = [hadamard_mpo(b[0]), hadamard_mpo(b[1])]
        # B_i(b) = sum_j 1/2 (b_j (.) D_j b_i + D_j (b_j (.) b_i)) - (1/Re) D_j^2 b_i,
        # entering the right-hand side with the weight -h (weight 1 when fitted)
        g = 1.0 if fit else -h
        for i in range(2):
            if not fit:
                rhs.append(Network(i, [], ('fixed', a[i]), 1.0))
            for j in range(2):
                rhs.append(Network(i, [H[j], D[j]], ('fixed', b[i]), 0.5 * g))
                rhs.append(Network(i, [D[j], H[j]], ('fixed', b[i]), 0.5 * g))
            rhs.append(Network(i, [Lap], ('fixed', b[i]), -g / prm.re))
    pen = {}
    if fit:
        return rhs, pen
    for i in range(2):
        for j in range(2):
            pen[(i, j)] = Network(i, [DT[i], D[j]], ('v', j), prm.mu * h * h)
    return rhs, pen


def cg(matvec, rhs, x0, rtol, maxit):
    """Conjugate gradients on the stacked vector; stops when the recursively
    updated residual satisfies ||r|| <= rtol ||rhs|| (Sec. II.C)."""
    bnorm = float(np.sqrt(rhs @ rhs))
    if bnorm == 0.0:
        return np.zeros_like(rhs), 0, True
    x = x0.copy()
    r = rhs - matvec(x)
    rr = float(r @ r)
    tol2 = (rtol * bnorm) ** 2
    if rr <= tol2:
        return x, 0, True
    p = r.copy()
    for it in range(1, maxit + 1):
        q = matvec(p)
        alpha = rr / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        if rr_new <= tol2:
            return x, it, True
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxit, False


def local_solve(d, v, rhs_nets, pen, prm, stats):
    shape = [v[0][d].shape, v[1][d].shape]
    sizes = [int(np.prod(s)) for s in shape]
    rhs = []
    for i in range(2):
        r = np.zeros(shape[i])
        for net in rhs_nets:
            if net.bra == i:
                r += net.coef * net.open(d, net.ket_core(v, d))
        rhs.append(r.reshape(-1))
    rhs = np.concatenate(rhs)

    def matvec(x):
        xs = [x[:sizes[0]].reshape(shape[0]), x[sizes[0]:].reshape(shape[1])]
        y = [xs[0].copy(), xs[1].copy()]
        for (i, j), net in pen.items():
            y[i] += net.coef * net.open(d, xs[j])
        return np.concatenate([y[0].reshape(-1), y[1].reshape(-1)])

    x0 = np.concatenate([v[0][d].reshape(-1), v[1][d].reshape(-1)])
    if not pen:
        # fit of B(b): the local matrix is the identity
        v[0][d] = rhs[:sizes[0]].reshape(shape[0])
        v[1][d] = rhs[sizes[0]:].reshape(shape[1])
        return
    x, its, ok = cg(matvec, rhs, x0, prm.cg_rtol, prm.cg_maxit)
    v[0][d] = x[:sizes[0]].reshape(shape[0])
    v[1][d] = x[sizes[0]:].reshape(shape[1])
    stats.cg_iters_total += its
    stats.cg_iters_max = max(stats.cg_iters_max, its)
    stats.cg_solves += 1
    stats.cg_maxit_hits += 0 if ok else 1


def project(a, b, h, prm, guess, stats=None):
    """argmin_v Theta(v; a, b, h) over MPS with the bonds of the guess
    (App. B).  Returns the two MPS with the centre at site 0.

    rhs_mode 1 (explicit right-hand side): B(b) is first fitted as one
    chi-bounded MPS w on the bonds of b (from the guess b, the same sweeps),
    then Theta is minimised with the right-hand side a - h w."""
    if stats is None:
        stats = Stats()
    if prm.rhs_mode == 1:
        w = sweep_fit(b, prm, [M.copy(b[0]), M.copy(b[1])])
        return _sweep(a, None, h, prm, guess, stats, w=w)
    return _sweep(a, b, h, prm, guess, stats)


def sweep_fit(b, prm, guess):
    """Least-squares fit of B(b) (Eq. MPS_momentum's convection and diffusion,
    App. B) on the bonds of the guess by the one-site sweep."""
    if prm.fit_sweeps > 0:
        prm = replace(prm, max_sweeps=prm.fit_sweeps)
    return _sweep(None, b, 0.0, prm, guess, Stats(), fit=True)


def _sweep(a, b, h, prm, guess, stats, w=None, fit=False):
    n = len(guess[0])
    v = [M.right_canonicalize(g) for g in guess]
    rhs_nets, pen = build_networks(a, b, h, prm, n, w=w, fit=fit)
    nets = rhs_nets + list(pen.values())
    for net in nets:
        net.init(v, n)
    nrm_prev = sum(float(np.sum(v[i][0] ** 2)) for i in range(2))
    for s in range(prm.max_sweeps):
        for d in range(0, n - 1):
            local_solve(d, v, rhs_nets, pen, prm, stats)
            for i in range(2):
                M.shift_right(v[i], d)
            for net in nets:
                net.update_left(v, d)
        for d in range(n - 1, 0, -1):
            local_solve(d, v, rhs_nets, pen, prm, stats)
            for i in range(2):
                M.shift_left(v[i], d)
            for net in nets:
                net.update_right(v, d)
        stats.sweeps += 1
        nrm = sum(float(np.sum(v[i][0] ** 2)) for i in range(2))
        if prm.sweep_rtol > 0.0 and abs(nrm - nrm_prev) <= prm.sweep_rtol * nrm:
            break
        nrm_prev = nrm
    return v


RK4_B_TABLE = [(3.0, 0.25), (1.5, 0.625), (3.0, 0.25)]
RK4_H = [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]


def rk4_step(u, prm, stats=None):
    """One RK4 step (App. B, Eqs. U1-U4); returns (u_new, per-stage stats)."""
    a = [M.scale(u[i], 0.25) for i in range(2)]
    U, st = [], []
    for k in range(4):
        if k == 0:
            b = [M.copy(u[0]), M.copy(u[1])]
        else:
            c, cu = RK4_B_TABLE[k - 1]
            b = [M.truncate(M.add([c, cu], [U[-1][i], u[i]]), prm.chi, prm.svd_rtol)[0]
                 for i in range(2)]
        s = Stats()
        U.append(project(a, b, RK4_H[k] * prm.dt, prm, a, s))
        st.append(s)
    new = [M.truncate(M.add([1.0] * 4, [U[k][i] for k in range(4)]), prm.chi,
                      prm.svd_rtol)[0] for i in range(2)]
    return new, st


def rk1_step(u, prm, stats=None):
    """One explicit Euler step (App. B, Eq. euler): argmin Theta(v; u, u, dt),
    from the guess u; returns (u_new, [stats])."""
    s = Stats()
    new = project([M.copy(u[0]), M.copy(u[1])], [M.copy(u[0]), M.copy(u[1])], prm.dt, prm,
                  [M.copy(u[0]), M.copy(u[1])], s)
    return new, [s]


def rk2_step(u, prm, stats=None):
    """One midpoint (RK2) step (App. B, Eqs. midpoint_calc, full_calc): the
    state at t + dt/2 from Theta(v; u, u, dt/2), then the full step from
    Theta(v; u, u_mid, dt), both from the guess u; returns (u_new, stats)."""
    a = [M.copy(u[0]), M.copy(u[1])]
    s1, s2 = Stats(), Stats()
    mid = project(a, a, 0.5 * prm.dt, prm, [M.copy(u[0]), M.copy(u[1])], s1)
    new = project(a, mid, prm.dt, prm, [M.copy(u[0]), M.copy(u[1])], s2)
    return new, [s1, s2]
