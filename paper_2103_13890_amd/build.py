"""Build libjfnk.so for gfx950 with hipcc (in-tree).

Each HIP translation unit under csrc/ compiles in parallel to an object in
_build/, then they are linked into paper_2103_13890_amd/libjfnk.so.
Run:  python -m paper_2103_13890_amd.build   (or build() from Python).
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
OUT = os.path.join(HERE, 'libjfnk.so')
BUILD = os.path.join(os.path.dirname(HERE), '_build')
ARCH = os.environ.get('JFNK_ARCH', 'gfx950')

# Packed FP32 instructions are disabled for every HIP object.
FLAGS = ['-O3', f'--offload-arch={ARCH}', '-std=c++17', '-fPIC', '-Wall',
         '-Wno-unused-function', '-Wno-unused-variable',
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops']

SOURCES = ['jfnk.hip', 'ops_f64.hip', 'ops_f32.hip', 'vec.hip', 'coarse.hip']


def _hipcc():
    path = shutil.which('hipcc') or '/opt/rocm/bin/hipcc'
    if not os.path.exists(path):
        raise RuntimeError('hipcc not found')
    return path


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + '.o')
    cmd = [_hipcc()] + FLAGS + ['-c', os.path.join(CSRC, src), '-o', obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'hipcc failed for {src}:\n{r.stderr}')
    warn = '\n'.join(l for l in r.stderr.splitlines() if 'packed-fp32-ops' not in l and l.strip())
    return obj, warn


def build(verbose=False):
    """Compile every HIP source for the target arch and link libjfnk.so."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    for _, warn in results:
        if verbose and warn:
            print(warn, file=sys.stderr)
    tmp = OUT + '.tmp'
    # the marker ranges of the host control (roctx, read by rocprofv3 --marker-trace)
    rocm_lib = os.path.join(os.environ.get('ROCM_PATH', '/opt/rocm'), 'lib')
    cmd = ([_hipcc(), f'--offload-arch={ARCH}', '-shared', '-fPIC', '-o', tmp] + [o for o, _ in results] +
           [f'-L{rocm_lib}', f'-Wl,-rpath,{rocm_lib}', '-lrocprofiler-sdk-roctx'])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError('link failed:\n' + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == '__main__':
    print(build(verbose=True))
