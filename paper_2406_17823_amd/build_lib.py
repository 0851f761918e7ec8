"""Build libqtt.so (HIP, gfx950) in-tree from csrc/*.hip.

Every call compiles from source; objects go to csrc/_build/ and the shared
library to the package directory, where the Python binding loads it.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
OUT = os.path.join(HERE, 'libqtt.so')
ARCH = os.environ.get('QTT_OFFLOAD_ARCH', 'gfx950')
FLAGS = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}',
         # packed fp32 instructions are disabled for all device code
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
         '-I', os.path.join(HERE, '..', 'include')]


def _compile(src, obj):
    cmd = ['hipcc', *FLAGS, '-c', src, '-o', obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = '\n'.join(l for l in r.stderr.splitlines() if 'packed-fp32-ops' not in l)
    if r.returncode != 0:
        raise RuntimeError(f'hipcc failed for {src}:\n{err}')
    return obj


def build(verbose=False):
    bdir = os.path.join(CSRC, '_build')
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, '*.hip')))
    objs = [os.path.join(bdir, os.path.basename(s)[:-4] + '.o') for s in srcs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        list(ex.map(_compile, srcs, objs))
    tmp = OUT + '.tmp'
    cmd = ['hipcc', f'--offload-arch={ARCH}', '-shared', '-fPIC', *objs, '-o', tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError('link failed:\n' + r.stderr)
    os.replace(tmp, OUT)
    if verbose:
        print('built', OUT)
    return OUT


if __name__ == '__main__':
    build(verbose=True)
    sys.exit(0)
