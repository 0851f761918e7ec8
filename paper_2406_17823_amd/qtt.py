"""Python binding of libqtt.so (argument marshalling only).

Every operation runs in the HIP library; this module only converts torch
device tensors and Python lists to the C descriptors of include/qtt.h.
Importing it on a machine without the built library raises immediately.
"""
import ctypes
import os

import numpy as np
import torch

MAX_SITES = 16
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libqtt.so')

PREC_F64, PREC_F32, PREC_BF16X3 = 0, 1, 2
PC_NONE, PC_BLOCK_JACOBI, PC_LEARNED = 0, 1, 2
W_CG_MAXIT, W_SWEEP_MAXIT, W_PRECOND_FALLBACK, W_SVD_MAXIT = 1, 2, 3, 4
ERRORS = {-1: 'QTT_E_ARG', -2: 'QTT_E_SHAPE', -3: 'QTT_E_CAPACITY', -4: 'QTT_E_HIP',
          -5: 'QTT_E_NAN', -6: 'QTT_E_UNSUPPORTED'}


class c_mps(ctypes.Structure):
    _fields_ = [('n', ctypes.c_int32), ('bond', ctypes.c_int32 * (MAX_SITES + 1)),
                ('capacity', ctypes.c_int64), ('data', ctypes.c_void_p)]


class c_mpo(ctypes.Structure):
    _fields_ = [('n', ctypes.c_int32), ('bond', ctypes.c_int32 * (MAX_SITES + 1)),
                ('capacity', ctypes.c_int64), ('data', ctypes.c_void_p)]


class c_params(ctypes.Structure):
    _fields_ = [('re', ctypes.c_double), ('dt', ctypes.c_double), ('mu', ctypes.c_double),
                ('dx', ctypes.c_double), ('chi', ctypes.c_int32), ('svd_rtol', ctypes.c_double),
                ('cg_rtol', ctypes.c_double), ('cg_maxit', ctypes.c_int32),
                ('sweep_rtol', ctypes.c_double), ('max_sweeps', ctypes.c_int32),
                ('lap_mode', ctypes.c_int32), ('prec', ctypes.c_int32), ('precond', ctypes.c_int32),
                ('rhs_mode', ctypes.c_int32), ('fit_sweeps', ctypes.c_int32)]


class c_stats(ctypes.Structure):
    _fields_ = [('sweeps', ctypes.c_int32 * 4), ('cg_iters_total', ctypes.c_int32),
                ('cg_iters_max', ctypes.c_int32), ('cg_solves', ctypes.c_int32),
                ('cg_maxit_hits', ctypes.c_int32), ('fallbacks', ctypes.c_int32),
                ('graph_replays', ctypes.c_int32),
                ('discarded_sq', ctypes.c_double), ('phase_ms', ctypes.c_double * 8)]

    def as_dict(self):
        return dict(sweeps=list(self.sweeps), cg_iters_total=self.cg_iters_total,
                    cg_iters_max=self.cg_iters_max, cg_solves=self.cg_solves,
                    cg_maxit_hits=self.cg_maxit_hits, fallbacks=self.fallbacks,
                    graph_replays=self.graph_replays,
                    discarded_sq=self.discarded_sq, phase_ms=list(self.phase_ms))


class c_kstats(ctypes.Structure):
    _fields_ = [('launches', ctypes.c_int64), ('timed', ctypes.c_int64),
                ('flops', ctypes.c_double), ('timed_ms', ctypes.c_double)]


SYMBOLS = ['qtt_kernel_timing', 'qtt_kernel_stats_read', 'qtt_ctx_create', 'qtt_ctx_destroy', 'qtt_last_error', 'qtt_mps_size',
           'qtt_mpo_derivative', 'qtt_add', 'qtt_truncate', 'qtt_apply_mpo', 'qtt_hadamard',
           'qtt_inner', 'qtt_to_dense', 'qtt_from_dense', 'qtt_project', 'qtt_rk4_step',
           'qtt_precond_config', 'qtt_precond_info', 'qtt_precond_weights', 'qtt_precond_grad',
           'qtt_rk4_step_batched', 'qtt_rk_step', 'qtt_schmidt_counts', 'qtt_dns_rhs',
           'qtt_dns_project', 'qtt_dns_step', 'qtt_fidelity', 'qtt_tke_shells', 'qtt_tke_spectrum',
           'qtt_inner_noalloc', 'qtt_precond_save', 'qtt_precond_load']

_lib = None


def lib():
    """The loaded libqtt.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f'libqtt.so not built ({LIB_PATH}); run __graft_entry__.build()')
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pm, pmo = ctypes.POINTER(c_mps), ctypes.POINTER(c_mpo)
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        'qtt_ctx_create': (I32, [ctypes.POINTER(P), I32, P]),
        'qtt_ctx_destroy': (None, [P]),
        'qtt_last_error': (ctypes.c_char_p, [P]),
        'qtt_mps_size': (I64, [I32, ctypes.POINTER(I32)]),
        'qtt_mpo_derivative': (I32, [P, I32, I32, I32, D, pmo]),
        'qtt_add': (I32, [P, I32, pd, pm, pm]),
        'qtt_truncate': (I32, [P, pm, I32, D, pd]),
        'qtt_apply_mpo': (I32, [P, pmo, pm, I32, D, pm, pd]),
        'qtt_hadamard': (I32, [P, pm, pm, I32, D, pm, pd]),
        'qtt_inner': (I32, [P, pm, pm, pd]),
        'qtt_inner_noalloc': (I32, [P, pm, pm, P]),
        'qtt_to_dense': (I32, [P, pm, P]),
        'qtt_from_dense': (I32, [P, P, I32, I32, D, pm]),
        'qtt_project': (I32, [P, pm, pm, D, ctypes.POINTER(c_params), pm,
                              ctypes.POINTER(c_stats)]),
        'qtt_rk4_step': (I32, [P, pm, ctypes.POINTER(c_params), ctypes.POINTER(c_stats)]),
        'qtt_rk_step': (I32, [P, pm, ctypes.POINTER(c_params), I32, ctypes.POINTER(c_stats)]),
        'qtt_schmidt_counts': (I32, [P, P, I32, ctypes.c_double, I32, ctypes.POINTER(I32)]),
        'qtt_dns_rhs': (I32, [P, P, P, P, P, I32, ctypes.c_double]),
        'qtt_dns_project': (I32, [P, P, P, I32]),
        'qtt_dns_step': (I32, [P, P, P, I32, ctypes.c_double, ctypes.c_double, I32, I32]),
        'qtt_fidelity': (I32, [P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
        'qtt_tke_shells': (I32, [I32]),
        'qtt_tke_spectrum': (I32, [P, P, P, P, P, I32, ctypes.POINTER(ctypes.c_double), I32]),
        'qtt_kernel_timing': (I32, [P, I32, I32]),
        'qtt_kernel_stats_read': (I32, [P, I32, ctypes.POINTER(c_kstats)]),
        'qtt_precond_config': (I32, [P, I32, D, ctypes.c_uint64, I32]),
        'qtt_precond_info': (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64), pd, pd]),
        'qtt_precond_weights': (I32, [P, I32, pd, I64]),
        'qtt_precond_save': (I32, [P, ctypes.c_char_p]),
        'qtt_precond_load': (I32, [P, ctypes.c_char_p]),
        'qtt_precond_grad': (I32, [P, P, I64, P, P, P]),
        'qtt_rk4_step_batched': (I32, [P, I32, pm, ctypes.POINTER(c_params),
                                       ctypes.POINTER(c_stats), I32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class QttError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'{ERRORS.get(code, code)}: {msg}')
        self.code = code


class Context:
    """One library context on a device, enqueuing on torch's current stream."""

    def __init__(self, device=0):
        L = lib()
        self.device = device
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        rc = L.qtt_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(stream))
        if rc != 0:
            raise QttError(rc, 'qtt_ctx_create failed')
        self.h = h
        self.last_warning = 0

    def close(self):
        if getattr(self, 'h', None):
            lib().qtt_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc, what):
        if rc < 0:
            msg = lib().qtt_last_error(self.h).decode()
            raise QttError(rc, f'{what}: {msg}')
        self.last_warning = rc
        return rc


def mps_size(bonds):
    return int(sum(bonds[k] * 4 * bonds[k + 1] for k in range(len(bonds) - 1)))


class MPS:
    """A device MPS: bonds [1, ..., 1] and a float64 torch tensor holding the
    packed cores (capacity >= the packed size)."""

    def __init__(self, bonds, data):
        self.bonds = list(int(b) for b in bonds)
        self.data = data
        assert data.dtype == torch.float64 and data.is_cuda

    @property
    def n(self):
        return len(self.bonds) - 1

    @property
    def size(self):
        return mps_size(self.bonds)

    @classmethod
    def empty(cls, bonds, capacity=None, device='cuda'):
        cap = mps_size(bonds) if capacity is None else int(capacity)
        return cls(bonds, torch.zeros(max(cap, 1), dtype=torch.float64, device=device))

    @classmethod
    def from_cores(cls, cores, capacity=None, device='cuda'):
        bonds = [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]
        flat = np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel() for c in cores])
        cap = flat.size if capacity is None else max(int(capacity), flat.size)
        t = torch.zeros(cap, dtype=torch.float64, device=device)
        t[:flat.size] = torch.from_numpy(flat).to(device)
        return cls(bonds, t)

    def cores(self):
        flat = self.data[:self.size].cpu().numpy()
        out, o = [], 0
        for k in range(self.n):
            l, r = self.bonds[k], self.bonds[k + 1]
            out.append(flat[o:o + l * 4 * r].reshape(l, 4, r).copy())
            o += l * 4 * r
        return out

    def struct(self):
        s = c_mps()
        s.n = self.n
        for k, b in enumerate(self.bonds):
            s.bond[k] = b
        s.capacity = self.data.numel()
        s.data = self.data.data_ptr()
        return s

    def take(self, s):
        self.bonds = [int(s.bond[k]) for k in range(s.n + 1)]


class MPO:
    def __init__(self, bonds, data):
        self.bonds = list(bonds)
        self.data = data

    def struct(self):
        s = c_mpo()
        s.n = len(self.bonds) - 1
        for k, b in enumerate(self.bonds):
            s.bond[k] = b
        s.capacity = self.data.numel()
        s.data = self.data.data_ptr()
        return s


def params(re, dt, chi, dx, mu=2.5e5, svd_rtol=1e-12, cg_rtol=1e-12, cg_maxit=1000,
           sweep_rtol=0.0, max_sweeps=2, lap_mode=0, prec=PREC_F64, precond=PC_NONE,
           rhs_mode=0, fit_sweeps=0):
    p = c_params()
    p.re, p.dt, p.mu, p.dx, p.chi = re, dt, mu, dx, chi
    p.svd_rtol, p.cg_rtol, p.cg_maxit = svd_rtol, cg_rtol, cg_maxit
    p.sweep_rtol, p.max_sweeps, p.lap_mode = sweep_rtol, max_sweeps, lap_mode
    p.prec, p.precond, p.rhs_mode, p.fit_sweeps = prec, precond, rhs_mode, fit_sweeps
    return p


# ---------------------------------------------------------------- operations
def mpo_derivative(ctx, n, axis, order, dx):
    data = torch.zeros(n * 144, dtype=torch.float64, device=f'cuda:{ctx.device}')
    s = c_mpo()
    s.capacity = data.numel()
    s.data = data.data_ptr()
    ctx.check(lib().qtt_mpo_derivative(ctx.h, n, axis, order, dx, ctypes.byref(s)),
              'mpo_derivative')
    return MPO([s.bond[k] for k in range(n + 1)], data)


def add(ctx, coefs, xs, y=None):
    k = len(xs)
    bonds = [1] + [sum(x.bonds[s] for x in xs) for s in range(1, xs[0].n)] + [1]
    if y is None:
        y = MPS.empty(bonds, device=xs[0].data.device)
    arr = (c_mps * k)(*[x.struct() for x in xs])
    co = (ctypes.c_double * k)(*[float(c) for c in coefs])
    ys = y.struct()
    ctx.check(lib().qtt_add(ctx.h, k, co, arr, ctypes.byref(ys)), 'add')
    y.take(ys)
    return y


def truncate(ctx, y, chi, svd_rtol=1e-12):
    ys = y.struct()
    disc = ctypes.c_double()
    ctx.check(lib().qtt_truncate(ctx.h, ctypes.byref(ys), chi, svd_rtol, ctypes.byref(disc)),
              'truncate')
    y.take(ys)
    return disc.value


def apply_mpo(ctx, W, x, chi=0, svd_rtol=1e-12, y=None):
    if y is None:
        y = MPS.empty([a * b for a, b in zip(W.bonds, x.bonds)], device=x.data.device)
    ws, xs, ys = W.struct(), x.struct(), y.struct()
    disc = ctypes.c_double()
    ctx.check(lib().qtt_apply_mpo(ctx.h, ctypes.byref(ws), ctypes.byref(xs), chi, svd_rtol,
                                  ctypes.byref(ys), ctypes.byref(disc)), 'apply_mpo')
    y.take(ys)
    return y, disc.value


def hadamard(ctx, a, b, chi=0, svd_rtol=1e-12, y=None):
    if y is None:
        y = MPS.empty([p * q for p, q in zip(a.bonds, b.bonds)], device=a.data.device)
    as_, bs, ys = a.struct(), b.struct(), y.struct()
    disc = ctypes.c_double()
    ctx.check(lib().qtt_hadamard(ctx.h, ctypes.byref(as_), ctypes.byref(bs), chi, svd_rtol,
                                 ctypes.byref(ys), ctypes.byref(disc)), 'hadamard')
    y.take(ys)
    return y, disc.value


def inner(ctx, x, y):
    out = ctypes.c_double()
    xs, ys = x.struct(), y.struct()
    ctx.check(lib().qtt_inner(ctx.h, ctypes.byref(xs), ctypes.byref(ys), ctypes.byref(out)),
              'inner')
    return out.value


def inner_noalloc(x, y, out, stream=None):
    """<x|y> into the device float64 tensor `out` (one element) without
    allocation, enqueued on `stream` (default: torch's current stream);
    returns the C return code (0, or QTT_E_* below zero)."""
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 1:
        raise ValueError('inner_noalloc: out must be a float64 device tensor')
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    xs, ys = x.struct(), y.struct()
    return lib().qtt_inner_noalloc(ctypes.c_void_p(stream.cuda_stream), ctypes.byref(xs),
                                   ctypes.byref(ys), ctypes.c_void_p(out.data_ptr()))


def to_dense(ctx, x):
    N = 1 << x.n
    g = torch.empty((N, N), dtype=torch.float64, device=x.data.device)
    xs = x.struct()
    ctx.check(lib().qtt_to_dense(ctx.h, ctypes.byref(xs), ctypes.c_void_p(g.data_ptr())),
              'to_dense')
    return g


def canonical_bonds(n, chi):
    return [1] + [min(chi, 4 ** k, 4 ** (n - k)) for k in range(1, n)] + [1]


def from_dense(ctx, grid, chi, svd_rtol=1e-12, capacity=None):
    N = grid.shape[0]
    n = N.bit_length() - 1
    cap = mps_size(canonical_bonds(n, chi)) if capacity is None else capacity
    out = MPS.empty(canonical_bonds(n, chi), capacity=cap, device=grid.device)
    g = grid.contiguous()
    os_ = out.struct()
    ctx.check(lib().qtt_from_dense(ctx.h, ctypes.c_void_p(g.data_ptr()), n, chi, svd_rtol,
                                   ctypes.byref(os_)), 'from_dense')
    out.take(os_)
    return out


def project(ctx, a, b, h, prm, v, stats=True):
    A = (c_mps * 2)(a[0].struct(), a[1].struct())
    B = (c_mps * 2)(b[0].struct(), b[1].struct())
    V = (c_mps * 2)(v[0].struct(), v[1].struct())
    st = c_stats()
    rc = ctx.check(lib().qtt_project(ctx.h, A, B, h, ctypes.byref(prm), V, ctypes.byref(st)),
                   'project')
    v[0].take(V[0])
    v[1].take(V[1])
    return rc, st.as_dict()


def rk4_step(ctx, u, prm):
    U = (c_mps * 2)(u[0].struct(), u[1].struct())
    st = c_stats()
    rc = ctx.check(lib().qtt_rk4_step(ctx.h, U, ctypes.byref(prm), ctypes.byref(st)), 'rk4_step')
    u[0].take(U[0])
    u[1].take(U[1])
    return rc, st.as_dict()


def rk_step(ctx, u, prm, order):
    """One step of the RK schedule of the given order (1: explicit Euler,
    2: midpoint, 4: RK4) in place on u; returns (code, stats dict)."""
    U = (c_mps * 2)(u[0].struct(), u[1].struct())
    st = c_stats()
    rc = ctx.check(lib().qtt_rk_step(ctx.h, U, ctypes.byref(prm), int(order), ctypes.byref(st)),
                   'rk_step')
    u[0].take(U[0])
    u[1].take(U[1])
    return rc, st.as_dict()


def schmidt_counts(ctx, grid, eps, chi_cap=256):
    """chi_l(eps) of every bipartition of a dense N x N float64 device grid
    (list of n - 1 ints)."""
    N = grid.shape[0]
    n = N.bit_length() - 1
    if tuple(grid.shape) != (N, N) or (1 << n) != N or grid.dtype != torch.float64:
        raise ValueError('schmidt_counts: N x N float64 grid with N a power of two')
    g = grid.contiguous()
    out = (ctypes.c_int32 * (n - 1))()
    ctx.check(lib().qtt_schmidt_counts(ctx.h, ctypes.c_void_p(g.data_ptr()), n, float(eps),
                                       int(chi_cap), out), 'schmidt_counts')
    return list(out)


def _grid_n(what, *gs):
    N = gs[0].shape[0]
    n = N.bit_length() - 1
    for g in gs:
        if (tuple(g.shape) != (N, N) or (1 << n) != N or g.dtype != torch.float64
                or not g.is_cuda or not g.is_contiguous()):
            raise ValueError(f'{what}: contiguous N x N float64 device grids, N a power of two')
    return n


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def dns_rhs(ctx, u1, u2, re):
    """C + D of the DNS at (u1, u2): returns two new grids."""
    n = _grid_n('dns_rhs', u1, u2)
    f1, f2 = torch.empty_like(u1), torch.empty_like(u2)
    ctx.check(lib().qtt_dns_rhs(ctx.h, _vp(u1), _vp(u2), _vp(f1), _vp(f2), n, float(re)),
              'dns_rhs')
    return f1, f2


def dns_project(ctx, u1, u2):
    """Divergence-free projection of (u1, u2), in place."""
    n = _grid_n('dns_project', u1, u2)
    ctx.check(lib().qtt_dns_project(ctx.h, _vp(u1), _vp(u2), n), 'dns_project')


def dns_step(ctx, u1, u2, re, dt, order=4, steps=1):
    """`steps` DNS steps (order 1: Euler, 4: RK4) of (u1, u2), in place."""
    n = _grid_n('dns_step', u1, u2)
    ctx.check(lib().qtt_dns_step(ctx.h, _vp(u1), _vp(u2), n, float(re), float(dt), int(order),
                                 int(steps)), 'dns_step')


def fidelity(ctx, a, b):
    """<a|b>^2 / (||a||^2 ||b||^2) of two float64 device tensors of one size."""
    if a.numel() != b.numel() or a.dtype != torch.float64 or b.dtype != torch.float64:
        raise ValueError('fidelity: two float64 device tensors of one size')
    a, b = a.contiguous(), b.contiguous()
    F = ctypes.c_double()
    ctx.check(lib().qtt_fidelity(ctx.h, _vp(a), _vp(b), a.numel(), ctypes.byref(F)), 'fidelity')
    return F.value


def tke_shells(n):
    return int(lib().qtt_tke_shells(int(n)))


def tke_spectrum(ctx, u1, u2, mean1=None, mean2=None):
    """E(k), k = 0 .. tke_shells(n) - 1, of u - mean (list of floats)."""
    gs = [u1, u2] + ([mean1, mean2] if mean1 is not None else [])
    n = _grid_n('tke_spectrum', *gs)
    S = tke_shells(n)
    E = (ctypes.c_double * max(S, 1))()
    ctx.check(lib().qtt_tke_spectrum(ctx.h, _vp(u1), _vp(u2), _vp(mean1), _vp(mean2), n, E, S),
              'tke_spectrum')
    return list(E)[:S]


def rk4_step_batched(ctx, flows, prms, workers=0):
    """One RK4 step of every flow (a list of [u1, u2] MPS pairs, updated in
    place) with its own parameters; returns (code, list of stats dicts)."""
    nf = len(flows)
    U = (c_mps * (2 * nf))(*[x.struct() for f in flows for x in f])
    Pp = (c_params * nf)(*prms)
    St = (c_stats * nf)()
    rc = ctx.check(lib().qtt_rk4_step_batched(ctx.h, nf, U, Pp, St, workers), 'rk4_step_batched')
    for f in range(nf):
        flows[f][0].take(U[2 * f])
        flows[f][1].take(U[2 * f + 1])
    return rc, [St[f].as_dict() for f in range(nf)]


def kernel_timing(ctx, enable=True, sample_every=1):
    ctx.check(lib().qtt_kernel_timing(ctx.h, 1 if enable else 0, sample_every), 'kernel_timing')


KERNEL_GEMM_F64_T64, KERNEL_GEMM_F32_T64, KERNEL_GEMM_F64_T128, KERNEL_GEMM_F32_T128 = 0, 1, 2, 3
# timed GEMM kinds; each is a family of instantiations that differ only in the
# operands' storage types (k_gemm<T, BM, BN, WGM, WGN, KD, SA, SB>)
KERNEL_NAMES = {0: 'k_gemm<double, 64, 64, 2, 2, 16, *>', 1: 'k_gemm<float, 64, 64, 2, 2, 16, *>',
                2: 'k_gemm<double, 128, 128, 2, 4, 32, *>',
                3: 'k_gemm<float, 128, 128, 2, 4, 32, *>'}


def kernel_stats(ctx, kernel):
    """Launch count, timed launches, executed flops and event time of one GEMM
    instantiation (KERNEL_GEMM_*) in the current timing window."""
    s = c_kstats()
    ctx.check(lib().qtt_kernel_stats_read(ctx.h, kernel, ctypes.byref(s)), 'kernel_stats_read')
    return dict(launches=s.launches, timed=s.timed, flops=s.flops, timed_ms=s.timed_ms)


PC_IN, PC_WIDTH, PC_OUT = 16, 256, 10


def precond_config(ctx, train_per_solve=0, lr=1e-3, seed=0x5eed, reset=False):
    ctx.check(lib().qtt_precond_config(ctx.h, train_per_solve, lr, seed, 1 if reset else 0),
              'precond_config')


def precond_info(ctx):
    n, s = ctypes.c_int64(), ctypes.c_int64()
    f, l = ctypes.c_double(), ctypes.c_double()
    ctx.check(lib().qtt_precond_info(ctx.h, ctypes.byref(n), ctypes.byref(s), ctypes.byref(f),
                                     ctypes.byref(l)), 'precond_info')
    return dict(nparam=n.value, steps=s.value, first_loss=f.value, last_loss=l.value)


def precond_weights(ctx, w=None):
    """Return the parameters (float64 numpy array), or set them when w is given."""
    import numpy as np
    n = precond_info(ctx)['nparam']
    if w is None:
        out = np.zeros(n)
        ctx.check(lib().qtt_precond_weights(ctx.h, 0, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), n), 'precond_weights')
        return out
    w = np.ascontiguousarray(w, dtype=np.float64)
    ctx.check(lib().qtt_precond_weights(ctx.h, 1, w.ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), w.size), 'precond_weights')
    return w


def precond_save(ctx, path):
    ctx.check(lib().qtt_precond_save(ctx.h, os.fsencode(path)), 'precond_save')


def precond_load(ctx, path):
    ctx.check(lib().qtt_precond_load(ctx.h, os.fsencode(path)), 'precond_load')


def precond_grad(ctx, X, dY):
    """Network output Y and gradient of sum(dY * Y) for device float64 X, dY."""
    assert X.dtype == torch.float64 and dY.dtype == torch.float64 and X.is_cuda and dY.is_cuda
    X, dY = X.contiguous(), dY.contiguous()
    npos = X.shape[0]
    assert X.shape == (npos, PC_IN) and dY.shape == (npos, PC_OUT)
    n = precond_info(ctx)['nparam']
    Y = torch.empty(npos, PC_OUT, dtype=torch.float64, device=X.device)
    g = torch.empty(n, dtype=torch.float64, device=X.device)
    ctx.check(lib().qtt_precond_grad(ctx.h, ctypes.c_void_p(X.data_ptr()), npos,
                                     ctypes.c_void_p(dY.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                     ctypes.c_void_p(g.data_ptr())), 'precond_grad')
    return Y, g

