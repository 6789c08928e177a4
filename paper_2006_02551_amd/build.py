"""Build the HIP library ``libwdg.so`` in-tree for gfx950 with hipcc.

Usage: ``python -m paper_2006_02551_amd.build`` (also called by the package's
build entry point).  Every call recompiles all sources.

``python -m paper_2006_02551_amd.build --sanitize`` builds ``_build/sanitize/libwdg.so``: the host C++
sources (setup, ABI, schemes, batching, adjoint driver) instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: each sanitizer flag applies to the host pass), linked with
the uninstrumented device objects.  Load it with the sanitizer runtime preloaded
(``sanitizer_env()``) and ``WDG_LIBRARY`` pointing at it.
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
LIB = os.path.join(HERE, "libwdg.so")
ARCH = "gfx950"

SOURCES = ["refel.cpp", "mesh.cpp", "api.cpp", "adjoint.cpp", "batch.cpp", "pml_schemes.cpp", "trace.cpp", "kernels.hip",
           "kernels_mfma.hip", "kernels_adjoint.hip", "peak.hip", "noalloc.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-pthread", f"-I{os.path.join(HERE, '..', 'include')}"]
# Packed FP32 instructions are disabled for all device code.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast", "-munsafe-fp-atomics"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + COMMON
    if src.endswith(".hip"):
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


SAN_DIR = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libwdg.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def sanitizer_runtime() -> str:
    """The clang AddressSanitizer runtime matching hipcc's compiler."""
    res = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        if not cands:
            raise RuntimeError("clang AddressSanitizer runtime not found")
        path = cands[-1]
    return path


def sanitizer_env() -> dict:
    """Environment for a Python process that loads the sanitizer build."""
    env = dict(os.environ)
    env["LD_PRELOAD"] = sanitizer_runtime()
    env["WDG_LIBRARY"] = SAN_LIB
    # the interpreter itself is not instrumented: its allocations at exit are not leaks of the library
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(SAN_DIR, exist_ok=True)

    def comp(src):
        obj = os.path.join(SAN_DIR, os.path.splitext(src)[0] + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc()] + COMMON + DEVICE + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd = [hipcc()] + COMMON + SAN_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(comp, SOURCES))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-shared-libsan"] + SAN_FLAGS + \
          ["-o", SAN_LIB] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
