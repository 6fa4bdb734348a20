"""Build the gfx950 HIP library libqbmi.so in-tree with hipcc.

    python -m paper_1503_07157_amd.build            # build (always recompiles)
    python -m paper_1503_07157_amd.build --asan     # host-ASan build, libqbmi_asan.so

Every translation unit is compiled for gfx950 only.  Packed FP32 vector
instructions are disabled (`-target-feature -packed-fp32-ops`), MFMA
accumulators are kept in VGPR form, and the sketch generator is compiled
without floating-point contraction so its Box-Muller transform is exactly
the sequence of correctly rounded operations it spells out.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqbmi.so")
ASAN_LIB = os.path.join(HERE, "libqbmi_asan.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# roctx ranges (rocprofiler-sdk-roctx) around the factorisation and its steps
LINK = [f"-L{os.path.join(ROCM, 'lib')}", "-lrocprofiler-sdk-roctx",
        f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
# AddressSanitizer on the host code only (device code is not instrumented)
ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    f"-I{os.path.join(os.path.dirname(HERE), 'include')}",
]
PER_FILE = {
    "k_sketch.hip": ["-ffp-contract=off"],
}
SOURCES = ["k_sketch.hip", "k_gemm64.hip", "k_gemm_batched.hip", "k_gemm_lowp.hip", "k_orth.hip",
           "k_misc.hip", "qb_api.hip",
           "k_post.hip", "qb_batch.hip", "qb_adjoint.hip", "prof.hip", "k_sample_i8.hip"]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the ROCm toolchain is required to build libqbmi.so")
    return path


def _compile(src: str, asan: bool = False) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", "_asan.o" if asan else ".o"))
    cmd = [hipcc(), *COMMON, *(ASAN if asan else []), *PER_FILE.get(src, []), "-c",
           os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False, asan: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, asan), SOURCES))
    out = ASAN_LIB if asan else LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *(ASAN if asan else []), *objs,
           *LINK, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True, asan="--asan" in sys.argv[1:])
    sys.exit(0)
