"""Summaries of rocprofv3 output for the benchmark's profiles.

    python -m paper_2406_17823_amd.tracesum window TRACE_CSV BENCH_LOG PATH
        per-kernel time, calls and average duration inside the timed window
        of one benchmark path (the window markers bench.py logs), and the
        fraction of the window in which the GPU ran a kernel;

    python -m paper_2406_17823_amd.tracesum mfma COUNTER_CSV CLOCK_GHZ
        MFMA busy fraction per kernel family from a counter-collection run with
        SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE: busy cycles summed over
        the dispatches / (dispatch durations x clock x 1024 SIMDs);

    python -m paper_2406_17823_amd.tracesum bytes FETCH_CSV WRITE_CSV KERNEL COPY_MIB
        HBM bytes per dispatch of KERNEL (a name, or a GEMM family
        'k_gemm<T, BM, BN, WGM, WGN, KD, *>') from two counter-collection runs
        (FETCH_SIZE, WRITE_SIZE), each scaled by what the same counter reads
        for the calibration copy of COPY_MIB MiB (which reads and writes
        exactly that many bytes);

    python -m paper_2406_17823_amd.tracesum sq COUNTER_CSV CLOCK_GHZ KERNEL
        per-dispatch means of every counter in a counter-collection run for
        KERNEL (a name or a GEMM family), and each over the dispatches' cycles.
"""
import collections
import csv
import re
import sys


def _short(name):
    name = re.sub(r'^void ', '', name).replace('qtt::(anonymous namespace)::', '')
    depth, out = 0, []
    for ch in name:            # drop the argument list, keep template arguments
        if ch == '(' and depth == 0:
            break
        depth += ch == '<'
        depth -= ch == '>'
        out.append(ch)
    return ''.join(out).strip()


def _family(name):
    """GEMM instantiations differing only in operand storage types and the
    CG-operand and vector-load flags form one family,
    'k_gemm<T, BM, BN, WGM, WGN, KD, *>' (the library times them as one
    kind)."""
    return re.sub(r', (double|float), (double|float)(, (true|false))*>$', ', *>', name)


def _matches(name, kernel):
    return _short(name) == kernel or ('*' in kernel and _family(_short(name)) == kernel)


def _window(log, path):
    w0 = w1 = secs = None
    for line in open(log):
        m = re.search(rf'{path} timed window start ns (\d+)', line)
        if m:
            w0 = int(m.group(1))
        m = re.search(rf'{path} timed window end ns (\d+)', line)
        if m:
            w1 = int(m.group(1))
        m = re.search(rf"\[bench\] {path} \{{'seconds': ([0-9.]+)", line)
        if m:
            secs = float(m.group(1))
    return w0, w1, secs


def window(trace, log, path):
    rows = []
    with open(trace) as f:
        for d in csv.DictReader(f):
            rows.append((int(d['Start_Timestamp']), int(d['End_Timestamp']), d['Kernel_Name']))
    w0, w1, secs = _window(log, path)
    sel = [r for r in rows if w0 is not None and r[0] >= w0 and r[1] <= w1]
    how = 'window markers'
    if not sel:
        # the profiler's clock differs from the host's: the timed steps of
        # this path end the run, take the last `secs` of the trace
        end = max(r[1] for r in rows)
        w0, w1 = end - int(secs * 1e9), end
        sel = [r for r in rows if r[0] >= w0 and r[1] <= w1]
        how = f'last {secs:.3f} s of the trace'
    tot = collections.defaultdict(lambda: [0, 0.0])
    for s, e, n in sel:
        k = _short(n)
        tot[k][0] += 1
        tot[k][1] += (e - s) / 1e6
    busy, cur = 0, None
    for s, e, _ in sorted(sel):
        if cur is None or s > cur[1]:
            if cur:
                busy += cur[1] - cur[0]
            cur = [s, e]
        else:
            cur[1] = max(cur[1], e)
    if cur:
        busy += cur[1] - cur[0]
    span = (w1 - w0) / 1e6
    print(f'timed window of path {path} ({how}): {span:.1f} ms, {len(sel)} kernels, '
          f'GPU busy {busy / 1e6:.1f} ms ({100 * busy / 1e6 / span:.0f}%)')
    print(f'{"total ms":>10} {"calls":>8} {"avg us":>9}  kernel')
    for k, (c, ms) in sorted(tot.items(), key=lambda x: -x[1][1])[:25]:
        print(f'{ms:10.2f} {c:8d} {1e3 * ms / c:9.2f}  {k}')
    fam = collections.defaultdict(lambda: [0, 0.0])
    for k, (c, ms) in tot.items():
        if _family(k) != k:
            fam[_family(k)][0] += c
            fam[_family(k)][1] += ms
    if fam:
        print('GEMM families (all operand storage types):')
        for k, (c, ms) in sorted(fam.items(), key=lambda x: -x[1][1]):
            print(f'{ms:10.2f} {c:8d} {1e3 * ms / c:9.2f}  {k}')


def _counter(csvfile, counter):
    """Summed counter value per dispatch: {dispatch: (kernel, value)}."""
    per = {}
    with open(csvfile) as f:
        r = csv.DictReader(f)
        cols = r.fieldnames
        kcol = next(c for c in cols if c.lower() in ('kernel_name', 'kernel-name'))
        ncol = next(c for c in cols if c.lower() in ('counter_name', 'counter-name'))
        vcol = next(c for c in cols if c.lower() in ('counter_value', 'counter-value'))
        dcol = next(c for c in cols if 'dispatch' in c.lower() and 'id' in c.lower())
        for d in r:
            if d[ncol] != counter:
                continue
            key = d[dcol]
            k, v = per.get(key, (d[kcol], 0.0))
            per[key] = (k, v + float(d[vcol]))
    return per


def bytes_per_dispatch(fetch_csv, write_csv, kernel, copy_mib):
    copy_bytes = copy_mib * (1 << 20)
    out = {}
    for name, f in (('FETCH_SIZE', fetch_csv), ('WRITE_SIZE', write_csv)):
        per = _counter(f, name)
        # the calibration copy: the largest dispatch outside the library
        cal = max((v for k, v in per.values() if 'qtt::' not in k), default=0.0)
        vals = [v for k, v in per.values() if _matches(k, kernel)]
        if not vals or cal <= 0:
            print(f'{name}: no dispatches of {kernel} or no calibration copy')
            return
        scale = copy_bytes / cal
        out[name] = (len(vals), sum(vals) / len(vals), scale)
        print(f'{name}: {len(vals)} dispatches of {kernel}, mean {sum(vals) / len(vals):.1f} '
              f'counter units; calibration copy {cal:.1f} units for {copy_bytes} bytes '
              f'({scale:.2f} bytes/unit) -> {scale * sum(vals) / len(vals):.4g} bytes/dispatch')
    tb = sum(v[1] * v[2] for v in out.values())
    print(f'traffic_bytes_per_dispatch {tb:.6g}')


def mfma(counter_csv, clock_ghz):
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    with open(counter_csv) as f:
        for d in csv.DictReader(f):
            a = agg[_family(_short(d['Kernel_Name']))]
            if d['Counter_Name'] == 'GRBM_GUI_ACTIVE':
                a['dur_ns'] += float(d['End_Timestamp']) - float(d['Start_Timestamp'])
                a['n'] += 1
            a[d['Counter_Name']] += float(d['Counter_Value'])
    print(f'{"MFMA busy":>10} {"dispatches":>10} {"avg us":>8}  kernel family')
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1].get('SQ_VALU_MFMA_BUSY_CYCLES', 0))[:8]:
        if not a['dur_ns']:
            continue
        util = a['SQ_VALU_MFMA_BUSY_CYCLES'] / (a['dur_ns'] * clock_ghz * 1024)
        print(f'{100 * util:9.1f}% {int(a["n"]):10d} {a["dur_ns"] / a["n"] / 1e3:8.1f}  {k}')


def sq(counter_csv, clock_ghz, kernel):
    """Per-dispatch means of every counter in the file for one kernel family, and each as a
    fraction of the dispatches' cycles (duration x clock)."""
    agg = collections.defaultdict(float)
    seen = set()
    n = 0
    dur = 0.0
    with open(counter_csv) as f:
        for d in csv.DictReader(f):
            if not _matches(d['Kernel_Name'], kernel):
                continue
            key = d.get('Dispatch_Id', d.get('Correlation_Id'))
            if key not in seen:
                seen.add(key)
                n += 1
                dur += float(d['End_Timestamp']) - float(d['Start_Timestamp'])
            agg[d['Counter_Name']] += float(d['Counter_Value'])
    if not n:
        print(f'no dispatches of {kernel}')
        return
    cyc = dur * clock_ghz
    print(f'{kernel}: {n} dispatches, {dur / n / 1e3:.1f} us each, {cyc / n:.4g} cycles each')
    print(f'{"counter":>28} {"per dispatch":>14} {"/ cycles":>10}')
    for c, v in sorted(agg.items()):
        print(f'{c:>28} {v / n:14.5g} {v / cyc:10.4g}')


if __name__ == '__main__':
    mode = sys.argv[1]
    if mode == 'window':
        window(sys.argv[2], sys.argv[3], sys.argv[4])
    elif mode == 'mfma':
        mfma(sys.argv[2], float(sys.argv[3]))
    elif mode == 'sq':
        sq(sys.argv[2], float(sys.argv[3]), sys.argv[4])
    elif mode == 'bytes':
        bytes_per_dispatch(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]))
    else:
        raise SystemExit(__doc__)
