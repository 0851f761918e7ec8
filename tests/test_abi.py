"""The C-ABI library builds, loads and exports every function include/qtt.h
declares; the Python binding's struct layouts match the header's sizes.
No compute call is made (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'qtt.h')
LIB = os.path.join(ROOT, 'paper_2406_17823_amd', 'libqtt.so')


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    return sorted(set(re.findall(r'\b(qtt_[a-z0-9_]+)\s*\(', text)))


@pytest.fixture(scope='module')
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_2406_17823_amd import qtt
    assert sorted(qtt.SYMBOLS) == declared_functions()


def test_struct_layouts():
    from paper_2406_17823_amd import qtt
    # qtt_mps: int32 n, int32 bond[17], int64 capacity, pointer data
    assert ctypes.sizeof(qtt.c_mps) == 4 + 17 * 4 + 8 + 8
    assert qtt.c_mps.capacity.offset == 72
    # qtt_params: 4 doubles, int32 (+pad), double, double, int32 (+pad), double, 6 int32
    assert qtt.c_params.svd_rtol.offset == 40
    assert qtt.c_params.sweep_rtol.offset == 64
    assert qtt.c_params.rhs_mode.offset == 88
    assert qtt.c_params.fit_sweeps.offset == 92
    assert ctypes.sizeof(qtt.c_params) == 96
    assert qtt.c_stats.discarded_sq.offset == 40
    assert ctypes.sizeof(qtt.c_stats) == 40 + 8 + 64


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """sizeof / offsetof of the header's structs as a C compiler lays them
    out, against the binding's ctypes mirrors."""
    import shutil
    import subprocess
    from paper_2406_17823_amd import qtt
    cc = shutil.which('gcc') or shutil.which('cc')
    if cc is None:
        pytest.skip('no C compiler')
    src = tmp_path / 'layout.c'
    fields = {'qtt_params': [f[0] for f in qtt.c_params._fields_],
              'qtt_stats': [f[0] for f in qtt.c_stats._fields_],
              'qtt_mps': [f[0] for f in qtt.c_mps._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qtt.h"', 'int main(void) {']
    for st, fs in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ['  return 0;', '}']
    src.write_text('\n'.join(lines) + '\n')
    exe = tmp_path / 'layout'
    subprocess.run([cc, '-std=c11', '-I', os.path.join(ROOT, 'include'), str(src), '-o', str(exe)],
                   check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True,
                                                        capture_output=True, text=True)
               .stdout.splitlines())
    for st, ct in (('qtt_params', qtt.c_params), ('qtt_stats', qtt.c_stats),
                   ('qtt_mps', qtt.c_mps)):
        assert int(out[st]) == ctypes.sizeof(ct), st
        for f in fields[st]:
            assert int(out[f'{st}.{f}']) == getattr(ct, f).offset, (st, f)


def test_mps_size_no_device(lib):
    f = lib.qtt_mps_size
    f.restype = ctypes.c_int64
    bonds = (ctypes.c_int32 * 6)(1, 4, 16, 16, 4, 1)
    assert f(5, bonds) == 4 * 4 + 4 * 4 * 16 + 16 * 4 * 16 + 16 * 4 * 4 + 4 * 4
    assert f(0, bonds) == -1


def test_context_without_device_reports_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip('a GPU is present')
    h = ctypes.c_void_p()
    f = lib.qtt_ctx_create
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_void_p]
    assert f(ctypes.byref(h), 0, None) == -4   # QTT_E_HIP
