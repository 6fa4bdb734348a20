"""The host side of the library under AddressSanitizer: the C-ABI argument
checks (tests/test_abi.py) run again against libqbmi_asan.so, the same
sources built with -fsanitize=address on the host code, in a child process
with the ASan runtime preloaded.  Any invalid read or write, double free or
overflow in the argument, size and workspace paths aborts the child with
an ASan report.  No GPU is used (the checks run before any device work)."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1503_07157_amd")
ASAN_LIB = os.path.join(PKG, "libqbmi_asan.so")


def _asan_runtime():
    for clang in ("/opt/rocm/llvm/bin/clang", "clang"):
        try:
            out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                 capture_output=True, text=True, timeout=60).stdout.strip()
        except (OSError, subprocess.SubprocessError):
            continue
        if out and os.path.isfile(out):
            return out
    return None


def _stale():
    if not os.path.exists(ASAN_LIB):
        return True
    t = os.path.getmtime(ASAN_LIB)
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + [os.path.join(ROOT, "include", "qb.h")]
    return any(os.path.getmtime(f) > t for f in srcs)


def test_abi_argument_paths_under_host_asan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    if _stale():
        subprocess.run([sys.executable, "-m", "paper_1503_07157_amd.build", "--asan"], cwd=ROOT,
                       check=True, capture_output=True, timeout=600)
    env = dict(os.environ, LD_PRELOAD=rt, QB_LIBRARY=ASAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    probe = ("import paper_1503_07157_amd._lib as L; lib = L.load(); "
             "maps = open('/proc/self/maps').read(); "
             "assert 'libqbmi_asan.so' in maps and 'libclang_rt.asan' in maps; print('asan-loaded')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0 and "asan-loaded" in r.stdout, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr
