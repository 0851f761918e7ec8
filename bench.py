#!/usr/bin/env python3
"""RK4 steps/s of the QTT Navier-Stokes step on one MI355X.

Workload: 2048 x 2048 periodic grid (11 quantics sites, d = 4), bond
dimension chi = 128, decaying-jet shear layer (App. C of the paper) at
Re = 1e7, dt = 5e-5.  The state is compressed from the dense initial field
on the GPU, advanced `--warmup` untimed RK4 steps in float64 (the bonds grow
from the jet's low rank towards chi), and then every solver path advances the
same state `--steps` timed RK4 steps (each path in turn):
  * mixed: float32-MFMA contractions of the convection networks, float64 QR /
    SVD / CG residual / overlap term, learned-preconditioner setting as given
    by --precond;
  * f64:   every contraction in float64 MFMA, unpreconditioned CG;
  * bf16x3: the convection networks as compensated split-bfloat16 MFMA
    products with float32 accumulation (its CG stops at --bf16x3-cg-rtol).
Every minimisation sweeps until the paper's stop rule holds (Sec. II.C:
relative change of sum_i <v_i|v_i> over a full sweep at most 1e-5, at most
10 sweeps) unless --sweeps fixes the count.
`value` is the mixed path's steps/s; the line also carries the float64 path's
steps/s, the parity protocol (one step of each reduced-precision path from
the common float64 state every `--parity-every` timed steps, relative L2
error of the velocity field and of each component), the end-state
difference after the timed steps, the sweeps the stop rule takes, the
roofline of the dominant GEMM kernel (HIP events around sampled launches,
executed flops counted on the device), and the CPU oracle timed on a
bounded sample and scaled to a step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X dense MFMA peaks, TFLOP/s, by GEMM instantiation (float64 / float32)
PEAK = {0: 78.6, 1: 157.3, 2: 78.6, 3: 157.3}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=2)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--spinup', type=int, default=-1,
                    help='untimed float64 steps that develop the jet before warm-up; '
                         '-1: until the largest bond of both components reaches chi (at most 16)')
    ap.add_argument('--n', type=int, default=11)
    ap.add_argument('--chi', type=int, default=128)
    ap.add_argument('--field', default='jet', choices=['jet', 'spectrum'],
                    help='initial field: the decaying jet (App. C) or the random-phase '
                         'spectrum E(k) ~ k^4 exp(-2 (k/k0)^2) (seeded, divergence-free)')
    ap.add_argument('--k0', type=float, default=16.0)
    ap.add_argument('--seed', type=int, default=5)
    ap.add_argument('--re', type=float, default=1e7)
    ap.add_argument('--dt', type=float, default=5e-5)
    ap.add_argument('--sweeps', type=int, default=0,
                    help='0: the stop rule of the sweep (Sec. II.C: relative change of '
                         'sum <v_i|v_i> over a full sweep at most 1e-5, at most 10 sweeps); '
                         'S > 0: exactly S sweeps per minimisation')
    ap.add_argument('--cg-rtol', type=float, default=1e-10)
    ap.add_argument('--mixed-cg-rtol', type=float, default=1e-9,
                    help='CG tolerance of the reduced-precision paths: their right-hand '
                         'sides carry float32 rounding of the convection terms (about 1e-10 '
                         'of the norm on this workload, the derivative MPO entries scale as '
                         '1/dx), so a tighter solve mostly fits that rounding')
    ap.add_argument('--bf16x3-cg-rtol', type=float, default=1e-8,
                    help='CG tolerance of the split-bfloat16 path: its convection operands '
                         'carry about 16 significant bits, and its step differs from the '
                         'float64 step by about 2e-8 whether CG stops at 1e-8 or 1e-9, so the '
                         'tighter solve only fits that rounding')
    ap.add_argument('--cg-maxit', type=int, default=1000)
    ap.add_argument('--paths', default='mixed,f64,bf16x3',
                    help='mixed: float32 convection networks; bf16x3: compensated split '
                         'bfloat16 convection networks; f64: all float64')
    ap.add_argument('--precond', type=int, default=0)
    ap.add_argument('--parity-every', type=int, default=20,
                    help='parity protocol: one step of each reduced-precision path from the '
                         'common float64 state at timed steps 0, E, 2E, ... (relative L2 per '
                         'component against the float64 step from the same state)')
    ap.add_argument('--sweep-rule', type=int, default=1,
                    help='also run one float64 step with the stop rule of the sweep (relative '
                         'change of sum <v_i|v_i> below 1e-5, at most 10 sweeps) and report the '
                         'sweeps it takes per stage next to the fixed count')
    ap.add_argument('--sample-every', type=int, default=8)
    ap.add_argument('--cpu-sample', type=int, default=1, help='time the CPU oracle sample')
    ap.add_argument('--save-state', default='', help='write the state after warm-up (.npz)')
    ap.add_argument('--load-state', default='', help='start from a saved state (no spin-up)')
    ap.add_argument('--schedules', default='',
                    help='also time the RK1 / RK2 schedules (e.g. "1,2") of every path from '
                         'the same state; reported under "schedules" with the relative L2 '
                         'difference to the float64 RK4 result after the same steps')
    ap.add_argument('--explicit-rhs', type=int, default=0,
                    help='also time RK4 with the explicit right-hand side (B(b) fitted as one '
                         'chi-bounded MPS in this many sweeps, then the minimisations) for every '
                         'path; reported under "explicit_rhs" with the difference to the '
                         'float64 implicit step')
    ap.add_argument('--schmidt', type=float, default=0.0,
                    help='also run the bond-dimension analysis chi_l(eps) at this eps on the '
                         'jet and spectrum initial fields and the developed state (GPU), with '
                         'the CPU oracle timed on the jet field; reported under "schmidt"')
    ap.add_argument('--dns', type=int, default=0,
                    help='also time this many RK4 steps of the dense DNS reference on the '
                         'decaying jet at the same size, Re and dt (GPU), compare it with the '
                         'tensor-network state at the same time by fidelity and TKE spectrum, '
                         'and time one step of the CPU oracle; reported under "dns"')
    ap.add_argument('--crossover', type=int, default=0,
                    help='also time one RK4 step of the tensor-network path (mixed and float64, '
                         'chi = 64) and of the dense DNS on the random-phase spectrum field for '
                         'n = 6 .. this value (at most 11), the runtime comparison over grid '
                         'sizes; reported under "crossover"')
    ap.add_argument('--learned', type=int, default=0,
                    help='also time this many RK4 steps of the mixed path with the learned '
                         'preconditioner (trained on-line on the solves\' own local systems, '
                         '--learned-train Adam steps per solve) from the same state; reported '
                         'under "learned" with CG iterations, fallbacks and the difference to '
                         'the float64 path')
    ap.add_argument('--learned-train', type=int, default=4)
    ap.add_argument('--batch', type=int, default=0,
                    help='also time this many RK4 steps of the batch of 64 independent flows '
                         'of uneven size (grids 2^8..2^11, chi 16..128, shear layers and '
                         'random-phase spectra, Re 1e4..1e6, dt = 0.2 / N, float32 convection '
                         'networks), batched on worker streams against one flow after another; '
                         'reported under "batch" in flow-steps/s')
    ap.add_argument('--batch-workers', type=int, default=8)
    ap.add_argument('--calib-copy-mib', type=int, default=0,
                    help='run one device-to-device copy of this many MiB before the timed '
                         'steps (reference dispatch for hardware byte counters)')
    return ap.parse_args()


def workload_name(args, n, chi):
    """The workload string of the JSON line's config (also the key of the
    byte-counter profiles)."""
    field = ('decaying jet' if args.field == 'jet' else
             f'random-phase spectrum (k0 = {args.k0:g}, seed {args.seed})')
    return (f'{field}, {1 << n}x{1 << n} grid ({n} sites), '
            f'chi={chi}, Re={args.re:g}, dt={args.dt:g}')


def measured_traffic(kernel, workload):
    """HBM bytes per dispatch of `kernel` on `workload` from the committed
    byte-counter profile, or None when there is none for this workload or
    the kernel source has changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, 'paper_2406_17823_amd', 'csrc', 'k_gemm.hip')
    sha = hashlib.sha256(open(src, 'rb').read()).hexdigest()[:16]
    for f in glob.glob(os.path.join(ROOT, 'profiles', '*_traffic.txt')):
        kv = {}
        for line in open(f):
            if ':' in line and not line.startswith(' '):
                k, v = line.split(':', 1)
                kv[k.strip()] = v.strip()
        if (kv.get('kernel') == kernel and kv.get('workload') == workload
                and kv.get('source', '').endswith(sha)):
            return float(kv['traffic_bytes_per_dispatch'])
    return None


def measured_cpu_step():
    """The committed timing of one complete oracle RK4 step at this size
    (profiles/cpu_oracle_rk4_step_*.txt), as a check of the sample's
    scaling, or None."""
    import glob
    for f in sorted(glob.glob(os.path.join(ROOT, 'profiles', 'cpu_oracle_rk4_step_*.txt'))):
        kv = {}
        for line in open(f):
            if ':' in line and not line.startswith(' '):
                k, v = line.split(':', 1)
                kv[k.strip()] = v.strip()
        if 'seconds_per_step' in kv:
            return dict(file=os.path.relpath(f, ROOT), seconds_per_step=float(kv['seconds_per_step']),
                        cores=int(kv.get('cores', 0)), workload=kv.get('workload', ''),
                        sample_seconds=float(kv.get('sample_seconds', 'nan')))
    return None


def log(*a):
    print('[bench]', *a, file=sys.stderr, flush=True)


def clone(Q, m):
    return Q.MPS(list(m.bonds), m.data.clone())


def sq_diff(Q, ctx, x, y, chi):
    """(||x - y||^2, ||y||^2) of one component; the difference is brought to
    canonical form first (its norm is then its centre's), which avoids the
    cancellation of <x|x> + <y|y> - 2<x|y>."""
    d = Q.add(ctx, [1.0, -1.0], [x, y])
    Q.truncate(ctx, d, 4 * chi, 0.0)     # canonical form; keeps every direction
    return max(Q.inner(ctx, d, d), 0.0), max(Q.inner(ctx, y, y), 0.0)


def rel_err(Q, ctx, X, Y, chi):
    """Relative L2 error of the velocity field X = (x1, x2) against Y:
    ||X - Y|| / ||Y|| over both components, and per component."""
    sq = [sq_diff(Q, ctx, X[i], Y[i], chi) for i in range(2)]
    field = (sum(d for d, _ in sq) / sum(y for _, y in sq)) ** 0.5
    return dict(field=field, components=[(d / y) ** 0.5 for d, y in sq])


def cpu_sample(uc, chi, re, dt):
    """Oracle right-environment build of one projection stage (all 20
    networks, sites n-1..1) on the benchmark's own state uc (two lists of
    float64 cores), as the first RK4 stage builds it."""
    from oracle import mps as M
    from oracle import sweep as S
    n = len(uc[0])
    a = [M.scale(c, 0.25) for c in uc]
    prm = S.Params(re=re, dt=dt, chi=chi, dx=1.0 / (1 << n))
    v = [M.right_canonicalize(x) for x in a]
    rhs, pen = S.build_networks(a, uc, dt / 6, prm, n)
    t0 = time.perf_counter()
    for net in rhs + list(pen.values()):
        net.init(v, n)
    t = time.perf_counter() - t0
    return t, threads_used()


def threads_used():
    """Host threads the oracle's BLAS calls can use."""
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    threads = int(os.environ.get('OMP_NUM_THREADS', cores))
    return min(threads, cores)


def main():
    args = parse()
    if args.gpus != 1:
        print(f'bench.py runs on one GPU only; --gpus {args.gpus} is not supported '
              '(the QTT step is not sharded across GPUs)', flush=True)
        sys.exit(2)
    import torch
    from paper_2406_17823_amd import inputs as I
    from paper_2406_17823_amd import qtt as Q

    n, chi = args.n, args.chi
    dx = 1.0 / (1 << n)
    ctx = Q.Context(0)
    cap = Q.mps_size(Q.canonical_bonds(n, chi))
    t0 = time.perf_counter()
    if args.load_state:
        import numpy as np
        z = np.load(args.load_state)
        state = []
        for c in range(2):
            bonds = [int(b) for b in z[f'bonds{c}']]
            st_ = Q.MPS.empty(bonds, capacity=cap)
            st_.data[:z[f'data{c}'].size] = torch.from_numpy(z[f'data{c}']).cuda()
            state.append(st_)
        args.spinup = 0
    else:
        u0 = I.decaying_jet(n) if args.field == 'jet' else I.spectrum(n, args.seed, k0=args.k0)
        state = [Q.from_dense(ctx, torch.from_numpy(u0[c]).cuda(), chi, 1e-12, capacity=cap)
                 for c in range(2)]
    log('initial bonds', state[0].bonds, state[1].bonds, f'{time.perf_counter() - t0:.1f}s')

    def prm_for(path, rhs_mode=0, fit_sweeps=0):
        return Q.params(re=args.re, dt=args.dt, chi=chi, dx=dx,
                        cg_rtol={'f64': args.cg_rtol, 'bf16x3': args.bf16x3_cg_rtol}.get(
                            path, args.mixed_cg_rtol),
                        cg_maxit=args.cg_maxit, max_sweeps=args.sweeps or 10,
                        sweep_rtol=0.0 if args.sweeps else 1e-5, svd_rtol=1e-12,
                        prec={'mixed': Q.PREC_F32, 'bf16x3': Q.PREC_BF16X3}.get(path, Q.PREC_F64),
                        precond=args.precond if path != 'f64' else Q.PC_NONE, rhs_mode=rhs_mode,
                        fit_sweeps=fit_sweeps)

    # spin-up: the jet starts with low QTT rank; the workload is the developed
    # flow whose bonds have reached chi (the paper times steps from t = 1)
    spin = 0
    limit = 16 if args.spinup < 0 else args.spinup
    while spin < limit:
        if args.spinup < 0 and min(max(state[0].bonds), max(state[1].bonds)) >= chi:
            break
        t1 = time.perf_counter()
        rc, st = Q.rk4_step(ctx, state, prm_for('f64'))
        torch.cuda.synchronize()
        spin += 1
        log(f'spin-up {spin} {time.perf_counter() - t1:.2f}s bonds', state[0].bonds,
            state[1].bonds, 'cg', st['cg_iters_total'], st['cg_iters_max'])

    for w in range(args.warmup):
        t1 = time.perf_counter()
        rc, st = Q.rk4_step(ctx, state, prm_for('f64'))
        torch.cuda.synchronize()
        log(f'warmup {w} {time.perf_counter() - t1:.2f}s bonds', state[0].bonds, state[1].bonds,
            'cg', st['cg_iters_total'], st['cg_iters_max'])

    if args.save_state:
        import numpy as np
        sz = [Q.mps_size(x.bonds) for x in state]
        np.savez(args.save_state, bonds0=np.array(state[0].bonds), bonds1=np.array(state[1].bonds),
                 data0=state[0].data[:sz[0]].cpu().numpy(), data1=state[1].data[:sz[1]].cpu().numpy())
    if args.calib_copy_mib > 0:
        nel = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device='cuda')
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f'calibration copy of {args.calib_copy_mib} MiB done')
        del src, dst

    paths = [p for p in args.paths.split(',') if p]
    results, finals, kstats = {}, {}, {}
    snaps = []   # (k, float64 state before timed step k, float64 state after it)
    for path in paths:
        prm = prm_for(path)
        # one untimed step of this path (its GEMM tile tuning, graph capture
        # and workspace growth happen here), then the timed steps from the
        # common state
        w = [clone(Q, state[0]), clone(Q, state[1])]
        Q.rk4_step(ctx, w, prm)
        del w
        u = [clone(Q, state[0]), clone(Q, state[1])]
        Q.kernel_timing(ctx, True, args.sample_every)
        cg_total, cg_solves = 0, 0
        sweeps_used = []
        torch.cuda.synchronize()
        log(f'{path} timed window start ns {time.monotonic_ns()}')
        t1 = time.perf_counter()
        for s in range(args.steps):
            snap = path == 'f64' and args.parity_every > 0 and s % args.parity_every == 0
            if snap:
                before = [clone(Q, u[0]), clone(Q, u[1])]
            rc, st = Q.rk4_step(ctx, u, prm)
            if snap:
                snaps.append((s, before, [clone(Q, u[0]), clone(Q, u[1])]))
            cg_total += st['cg_iters_total']
            cg_solves += st['cg_solves']
            sweeps_used.append(list(st['sweeps']))
            log(f'{path} step {s} {time.perf_counter() - t1:.2f}s cg {st["cg_iters_total"]} '
                f'sweeps {st["sweeps"]}')
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        log(f'{path} timed window end ns {time.monotonic_ns()}')
        kstats[path] = {k: Q.kernel_stats(ctx, k) for k in Q.KERNEL_NAMES}
        Q.kernel_timing(ctx, False)
        results[path] = dict(seconds=el, steps_per_s=args.steps / el,
                             cg_iters_per_solve=cg_total / max(cg_solves, 1),
                             cg_rtol=prm.cg_rtol,
                             sweeps_per_minimisation=sum(map(sum, sweeps_used)) /
                             max(4 * len(sweeps_used), 1))
        finals[path] = u
        log(path, results[path])

    main_path = 'mixed' if 'mixed' in results else paths[0]
    rel = None
    for p_ in results:
        if p_ != 'f64' and 'f64' in finals:
            e = rel_err(Q, ctx, finals[p_], finals['f64'], chi)
            results[p_]['rel_l2_vs_f64'] = e['field']
            results[p_]['rel_l2_vs_f64_components'] = e['components']
    if 'mixed' in results and 'f64' in finals:
        rel = results['mixed']['rel_l2_vs_f64']

    # parity protocol: every reduced-precision path takes one step from the
    # float64 state at timed steps 0, E, 2E, ... and is compared with the
    # float64 step from the same state; the end-state difference after all
    # timed steps (above) is reported beside it
    parity = None
    if snaps:
        parity = dict(bar=1e-5, every=args.parity_every,
                      protocol='one RK4 step of the path from the common float64 state at timed '
                               'steps 0, E, 2E, ...; relative L2 error of the velocity field '
                               '(both components) against the float64 step from that state, '
                               'and per component', paths={})
        for p_ in paths:
            if p_ == 'f64':
                continue
            errs, comps = [], []
            for k, before, after in snaps:
                w = [clone(Q, before[0]), clone(Q, before[1])]
                Q.rk4_step(ctx, w, prm_for(p_))
                e = rel_err(Q, ctx, w, after, chi)
                errs.append(e['field'])
                comps.append(e['components'])
            parity['paths'][p_] = dict(
                steps=[k for k, _, _ in snaps], per_step=errs, per_step_components=comps,
                per_step_max=max(errs), ok=max(errs) <= 1e-5,
                per_step_components_max=max(max(c) for c in comps),
                end_state_after_steps=args.steps, end_state=results[p_].get('rel_l2_vs_f64'),
                end_state_components=results[p_].get('rel_l2_vs_f64_components'))
            log('parity', p_, parity['paths'][p_])
        del snaps

    # the sweep's stop rule (Sec. II.C) at this workload: the sweeps it takes
    # per stage, and the float64 step it gives against two and three sweeps
    # from the same state
    sweep_rule = None
    if args.sweep_rule:
        w = [clone(Q, state[0]), clone(Q, state[1])]
        pr = prm_for('f64')
        pr.sweep_rtol, pr.max_sweeps = 1e-5, 10
        rc, st = Q.rk4_step(ctx, w, pr)
        sweep_rule = dict(sweep_rtol=1e-5, max_sweeps=10, sweeps_per_stage=list(st['sweeps']))
        for S_ in (2, 3):
            ref = [clone(Q, state[0]), clone(Q, state[1])]
            pr = prm_for('f64')
            pr.sweep_rtol, pr.max_sweeps = 0.0, S_
            Q.rk4_step(ctx, ref, pr)
            e = rel_err(Q, ctx, w, ref, chi)
            sweep_rule[f'rel_l2_rule_vs_{S_}_sweeps'] = e['field']
            sweep_rule[f'rel_l2_rule_vs_{S_}_sweeps_components'] = e['components']
        log('sweep rule', sweep_rule)

    learned = None
    if args.learned > 0:
        Q.precond_config(ctx, args.learned_train, 2e-3, 9, reset=True)
        prm = prm_for('mixed')
        prm.precond = Q.PC_LEARNED
        u = [clone(Q, state[0]), clone(Q, state[1])]
        cg_total, cg_solves, fb = 0, 0, 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.learned):
            rc, st = Q.rk4_step(ctx, u, prm)
            cg_total += st['cg_iters_total']
            cg_solves += st['cg_solves']
            fb += st['fallbacks']
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        info = Q.precond_info(ctx)
        learned = dict(steps=args.learned, steps_per_s=args.learned / el,
                       cg_iters_per_solve=cg_total / max(cg_solves, 1), fallbacks=fb,
                       train_per_solve=args.learned_train, probe_loss_first=info['first_loss'],
                       probe_loss_last=info['last_loss'],
                       plain_mixed_cg_iters_per_solve=results.get('mixed', {}).get('cg_iters_per_solve'),
                       plain_f64_steps_per_s=results.get('f64', {}).get('steps_per_s'))
        if 'f64' in finals and args.learned == args.steps:
            e = rel_err(Q, ctx, u, finals['f64'], chi)
            learned['rel_l2_vs_f64'] = e['field']
            learned['rel_l2_vs_f64_components'] = e['components']
        Q.precond_config(ctx, 0, 2e-3, 9)
        log('learned', learned)

    batch = None
    if args.batch > 0:
        import numpy as np
        specs = I.batch_flows()
        states, prms = [], []
        for f in specs:
            nf = f['n']
            g = (I.shear_layer(nf) if f['kind'] == 'shear' else
                 I.spectrum(nf, f['seed'], k0=8.0))
            capf = Q.mps_size(Q.canonical_bonds(nf, f['chi']))
            states.append([Q.from_dense(ctx, torch.from_numpy(np.ascontiguousarray(g[c])).cuda(),
                                        f['chi'], 1e-12, capacity=capf) for c in range(2)])
            prms.append(Q.params(re=f['re'], dt=f['dt'], chi=f['chi'], dx=1.0 / (1 << nf),
                                 cg_rtol=args.mixed_cg_rtol, cg_maxit=args.cg_maxit,
                                 max_sweeps=10, sweep_rtol=1e-5, svd_rtol=1e-12,
                                 prec=Q.PREC_F32))
        # untimed: one batched step grows every worker's workspace; the timed
        # runs start from the states after it
        Q.rk4_step_batched(ctx, states, prms, args.batch_workers)
        seq = [[clone(Q, x[0]), clone(Q, x[1])] for x in states]
        for f in range(len(seq)):
            Q.rk4_step(ctx, seq[f], prms[f])   # untimed: the main context's workspace
        seq = [[clone(Q, x[0]), clone(Q, x[1])] for x in states]
        bat = [[clone(Q, x[0]), clone(Q, x[1])] for x in states]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.batch):
            for f in range(len(seq)):
                Q.rk4_step(ctx, seq[f], prms[f])
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t1
        t1 = time.perf_counter()
        for _ in range(args.batch):
            Q.rk4_step_batched(ctx, bat, prms, args.batch_workers)
        torch.cuda.synchronize()
        t_bat = time.perf_counter() - t1
        same = all(bat[f][i].bonds == seq[f][i].bonds and
                   torch.equal(bat[f][i].data[:bat[f][i].size], seq[f][i].data[:seq[f][i].size])
                   for f in range(len(seq)) for i in range(2))
        nfl = len(seq)
        batch = dict(flows=nfl, steps=args.batch, workers=args.batch_workers,
                     flow_steps_per_s_batched=nfl * args.batch / t_bat,
                     flow_steps_per_s_sequential=nfl * args.batch / t_seq,
                     speedup=t_seq / t_bat, bitwise_equal_to_single_calls=same,
                     grids=sorted({1 << f['n'] for f in specs}),
                     chis=sorted({f['chi'] for f in specs}))
        log('batch', batch)
        del states, seq, bat

    schedules = None
    if args.schedules:
        schedules = {}
        for order in [int(x) for x in args.schedules.split(',') if x]:
            res = {}
            for path in paths:
                prm = prm_for(path)
                w = [clone(Q, state[0]), clone(Q, state[1])]
                Q.rk_step(ctx, w, prm, order)  # untimed: workspace growth, graphs
                del w
                u = [clone(Q, state[0]), clone(Q, state[1])]
                cg_total, cg_solves = 0, 0
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(args.steps):
                    rc, st = Q.rk_step(ctx, u, prm, order)
                    cg_total += st['cg_iters_total']
                    cg_solves += st['cg_solves']
                torch.cuda.synchronize()
                el = time.perf_counter() - t1
                r = dict(steps_per_s=args.steps / el, cg_iters_per_solve=cg_total / max(cg_solves, 1),
                         bonds=[u[0].bonds, u[1].bonds])
                if 'f64' in finals:
                    e = rel_err(Q, ctx, u, finals['f64'], chi)
                    r['rel_l2_vs_rk4_f64'] = e['field']
                    r['rel_l2_vs_rk4_f64_components'] = e['components']
                res[path] = r
                log(f'rk{order} {path}', r)
            schedules[f'rk{order}'] = res
        if 'f64' in finals:
            schedules['rk4_f64_bonds'] = [finals['f64'][0].bonds, finals['f64'][1].bonds]

    explicit = None
    if args.explicit_rhs:
        explicit = {}
        for path in paths:
            prm = prm_for(path, rhs_mode=1, fit_sweeps=args.explicit_rhs)
            w = [clone(Q, state[0]), clone(Q, state[1])]
            Q.rk4_step(ctx, w, prm)  # untimed: workspace growth, graphs
            del w
            u = [clone(Q, state[0]), clone(Q, state[1])]
            cg_total, cg_solves = 0, 0
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                rc, st = Q.rk4_step(ctx, u, prm)
                cg_total += st['cg_iters_total']
                cg_solves += st['cg_solves']
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            r = dict(steps_per_s=args.steps / el, cg_iters_per_solve=cg_total / max(cg_solves, 1))
            if 'f64' in finals:
                e = rel_err(Q, ctx, u, finals['f64'], chi)
                r['rel_l2_vs_implicit_f64'] = e['field']
                r['rel_l2_vs_implicit_f64_components'] = e['components']
            explicit[path] = r
            log(f'explicit rhs {path}', r)

    # roofline of the dominant kernel of the timed (value) path
    ks = kstats[main_path]

    def est_time(k):
        s = ks[k]
        return (s['timed_ms'] / s['timed'] * s['launches']) if s['timed'] else 0.0

    # the mixed path's dominant kernel is the float32 128-tile GEMM family
    # (largest share of GPU time in its kernel trace); HIP events bracket
    # every eighth launch and add a few microseconds of dispatch latency to
    # each bracketed launch, enough to reorder families of short kernels, so
    # the event totals pick the kernel only for the other paths
    dom = 3 if main_path == 'mixed' else max(Q.KERNEL_NAMES, key=est_time)
    s = ks[dom]
    avg_ms = s['timed_ms'] / max(s['timed'], 1)
    flops_per_launch = s['flops'] / max(s['launches'], 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    traffic = measured_traffic(Q.KERNEL_NAMES[dom], workload_name(args, n, chi))
    roofline = dict(bound='mfma', kernel=Q.KERNEL_NAMES[dom], achieved=round(achieved, 3),
                    peak=PEAK[dom], unit='TFLOP/s', frac=round(achieved / PEAK[dom], 4),
                    traffic=traffic, launches=s['launches'], avg_launch_ms=round(avg_ms, 5),
                    flops_per_launch=flops_per_launch,
                    kernel_share=round(est_time(dom) / (results[main_path]['seconds'] * 1e3), 3))

    dns = None
    if args.dns > 0:
        import numpy as np
        from oracle import dns as Dn
        N = 1 << n
        dj = I.decaying_jet(n)

        def jet():
            return [torch.from_numpy(np.ascontiguousarray(dj[c], dtype=np.float64)).cuda()
                    for c in range(2)]
        g = jet()
        Q.dns_step(ctx, g[0], g[1], args.re, args.dt, order=4, steps=1)  # untimed: workspace
        g = jet()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Q.dns_step(ctx, g[0], g[1], args.re, args.dt, order=4, steps=args.dns)
        torch.cuda.synchronize()
        t_dns = time.perf_counter() - t1
        # HBM bytes per grid point of one RK4 step as the kernels move them:
        # stage kernels 64 + 3 x 80, four projections of five 32-byte passes
        bpp = 64 + 3 * 80 + 4 * 160
        dns = dict(workload=f'decaying jet {N} x {N}, RK4, Re {args.re:g}, dt {args.dt:g}',
                   steps=args.dns, ms_per_step=round(1e3 * t_dns / args.dns, 3),
                   steps_per_s=round(args.dns / t_dns, 2), bytes_per_step=bpp * N * N,
                   achieved_GBps=round(bpp * N * N * args.dns / t_dns / 1e9, 1))
        log('dns', dns)
        if not args.load_state:
            # the tensor-network state is spin + warm-up steps after the jet
            k = spin + args.warmup
            g = jet()
            Q.dns_step(ctx, g[0], g[1], args.re, args.dt, order=4, steps=k)
            cmp = dict(steps=k, time=k * args.dt)
            for c in range(2):
                qd = Q.to_dense(ctx, state[c])
                cmp[f'fidelity_u{c + 1}'] = Q.fidelity(ctx, g[c], qd)
            Ed = np.array(Q.tke_spectrum(ctx, g[0], g[1]))
            Eq = np.array(Q.tke_spectrum(ctx, Q.to_dense(ctx, state[0]), Q.to_dense(ctx, state[1])))
            shells = [1, 4, 16, 64, 256, 1024]
            cmp['tke_shells'] = [s_ for s_ in shells if s_ < len(Ed)]
            cmp['tke_dns'] = [float(Ed[s_]) for s_ in cmp['tke_shells']]
            cmp['tke_qis'] = [float(Eq[s_]) for s_ in cmp['tke_shells']]
            dns['vs_tensor_network'] = cmp
            log('dns vs tensor network', cmp)
        # the oracle's RK4 step on the host, one step from the jet
        t1 = time.perf_counter()
        Dn.rk4_step([np.asarray(dj[0]), np.asarray(dj[1])], args.dt, args.re, 1.0 / N)
        dns['cpu_oracle'] = dict(seconds_per_step=round(time.perf_counter() - t1, 2),
                                 cores=threads_used())
        log('dns oracle', dns['cpu_oracle'])

    cross = None
    if args.crossover > 0:
        import numpy as np
        chi_x = 64
        cross = dict(chi=chi_x, field='random-phase spectrum (k0 = 8), compressed to chi',
                     rows=[])
        for nn in range(6, min(11, args.crossover) + 1):
            Nn = 1 << nn
            f = I.spectrum(nn, 2, k0=8.0)
            capn = Q.mps_size(Q.canonical_bonds(nn, chi_x))
            row = dict(n=nn)
            for path in ('mixed', 'f64'):
                pr = Q.params(re=args.re, dt=args.dt, chi=chi_x, dx=1.0 / Nn,
                              cg_rtol=args.cg_rtol if path == 'f64' else args.mixed_cg_rtol,
                              cg_maxit=args.cg_maxit, max_sweeps=args.sweeps or 10,
                              sweep_rtol=0.0 if args.sweeps else 1e-5, svd_rtol=1e-12,
                              prec=Q.PREC_F32 if path == 'mixed' else Q.PREC_F64)
                st_ = [Q.from_dense(ctx, torch.from_numpy(np.ascontiguousarray(f[c])).cuda(), chi_x,
                                    1e-12, capacity=capn) for c in range(2)]
                Q.rk4_step(ctx, st_, pr)  # untimed
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(2):
                    Q.rk4_step(ctx, st_, pr)
                torch.cuda.synchronize()
                row[f'qis_{path}_ms'] = round(1e3 * (time.perf_counter() - t1) / 2, 2)
                row['bonds_max'] = max(max(st_[0].bonds), max(st_[1].bonds))
            g = [torch.from_numpy(np.ascontiguousarray(f[c])).cuda() for c in range(2)]
            Q.dns_step(ctx, g[0], g[1], args.re, args.dt, order=4, steps=1)
            torch.cuda.synchronize()
            reps = 50
            t1 = time.perf_counter()
            Q.dns_step(ctx, g[0], g[1], args.re, args.dt, order=4, steps=reps)
            torch.cuda.synchronize()
            row['dns_ms'] = round(1e3 * (time.perf_counter() - t1) / reps, 4)
            cross['rows'].append(row)
            log('crossover', row)

    schmidt = None
    if args.schmidt > 0.0:
        eps = args.schmidt
        fields = {}
        dj, dt_ = I.decaying_jet(n), I.spectrum(n, 2, k0=8.0)
        for c in range(2):
            fields[f'jet u{c + 1}'] = torch.from_numpy(dj[c]).cuda()
            fields[f'spectrum u{c + 1}'] = torch.from_numpy(dt_[c]).cuda()
            fields[f'developed state u{c + 1}'] = Q.to_dense(ctx, state[c])
        schmidt = {'eps': eps, 'chi_cap': 256}
        for name, g in fields.items():
            Q.schmidt_counts(ctx, g, eps, chi_cap=256)  # untimed: workspace growth
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            cnt = Q.schmidt_counts(ctx, g, eps, chi_cap=256)
            torch.cuda.synchronize()
            schmidt[name] = dict(counts=cnt, chi=max(cnt),
                                 gpu_ms=round(1e3 * (time.perf_counter() - t1), 2))
            log('schmidt', name, schmidt[name])
        # the oracle's definition (one dense SVD per unfolding) on the jet's u1
        from oracle import schmidt as Sc
        t1 = time.perf_counter()
        ref = Sc.schmidt_counts(dj[0], eps)
        t_cpu = time.perf_counter() - t1
        cores = threads_used()
        schmidt['cpu_oracle'] = dict(field='jet u1', seconds=round(t_cpu, 3), cores=cores,
                                     counts_agree=(ref == schmidt['jet u1']['counts']))
        log('schmidt oracle', schmidt['cpu_oracle'])

    cpu = None
    if args.cpu_sample:
        # GPU time of the same sample (stage-1 environment build), phase-timed
        os.environ['QTT_TIMING'] = '1'
        tctx = Q.Context(0)
        os.environ.pop('QTT_TIMING')
        u = [clone(Q, state[0]), clone(Q, state[1])]
        prm = prm_for(main_path)
        prm.max_sweeps = 1
        a = [clone(Q, u[0]), clone(Q, u[1])]
        for x in a:
            x.data[:x.bonds[1] * 4] *= 0.25
        v = [clone(Q, a[0]), clone(Q, a[1])]
        rc, st = Q.project(tctx, a, u, args.dt / 6, prm, v)
        gpu_env_ms = st['phase_ms'][1]
        del tctx
        uc = [state[0].cores(), state[1].cores()]
        t_cpu, cores = cpu_sample(uc, chi, args.re, args.dt)
        step_s = results[main_path]['seconds'] / args.steps
        cpu_step_s = step_s * (t_cpu * 1e3) / max(gpu_env_ms, 1e-9)
        cpu = dict(value=round(1.0 / cpu_step_s, 6), unit='RK4 steps/s', cores=cores,
                   kind='oracle',
                   sample=(f'extrapolated from a timed sample: the oracle\'s right-environment '
                           f'build of the first RK4 stage (20 networks, sites {n - 1}..1) on the '
                           f'timed state ({1 << n}^2, chi={chi}) took {t_cpu:.1f} s on {cores} host '
                           f'threads against {gpu_env_ms:.1f} ms for the same phase on the GPU; '
                           f'the GPU step time is scaled by that ratio'))
        full = measured_cpu_step()
        if full is not None:
            cpu['full_step_measured'] = full

    line = dict(metric=f'RK4 steps/s, 2^{n}^2 grid chi={chi}, mixed vs FP64 plain at <=1e-5 rel L2 '
                       '(velocity field, one step from the common FP64 state)',
                value=round(results[main_path]['steps_per_s'], 5), unit='RK4 steps/s',
                n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=round(1e3 * results[main_path]['seconds'] / args.steps, 2),
                higher_is_better=True, scaling='weak', vs_baseline=None,
                dtype='f32' if main_path == 'mixed' else 'f64', data='synthetic',
                config=dict(workload=workload_name(args, n, chi),
                            spinup_steps=spin, bonds=[state[0].bonds, state[1].bonds],
                            sweeps=(args.sweeps if args.sweeps else
                                    'stop rule: relative change of sum <v_i|v_i> <= 1e-5, at most 10'),
                            cg_rtol=results[main_path]['cg_rtol'],
                            f64_cg_rtol=args.cg_rtol, precond=args.precond),
                paths={k: dict(v, **({} if k not in kstats else {})) for k, v in results.items()},
                rel_l2_mixed_vs_f64=rel, parity=parity, sweep_rule=sweep_rule,
                roofline=roofline, cpu_baseline=cpu)
    if learned is not None:
        line['learned'] = learned
    if batch is not None:
        line['batch'] = batch
    if schedules is not None:
        line['schedules'] = schedules
    if explicit is not None:
        line['explicit_rhs'] = explicit
    if schmidt is not None:
        line['schmidt'] = schmidt
    if dns is not None:
        line['dns'] = dns
    if cross is not None:
        line['crossover'] = cross
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == '__main__':
    main()
