"""Build the HIP library librpot.so for gfx950 in-tree.

    python -m paper_2311_15429_amd.build
    python -m paper_2311_15429_amd.build --sanitize   # librpot_san.so

The sanitizer build instruments the host code (planner, C-ABI, launch
set-up) with AddressSanitizer and UndefinedBehaviorSanitizer; device code is
built as usual.  It is for CPU runs of the host tests: load it with
RPOT_LIB=<path to librpot_san.so> and the sanitizer runtime first in
LD_PRELOAD (sanitizer_env() gives both).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librpot.so")
BUILD = os.path.join(HERE, "_build")
SAN_LIB = os.path.join(HERE, "librpot_san.so")
SAN_BUILD = os.path.join(HERE, "_build_san")

SOURCES = ["plan.cpp", "surrogate.cpp", "fft.hip", "fft_reg.hip", "lagsum.hip", "history.hip", "mlp.hip", "surrogate.hip",
           "coupling.hip", "calib.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-result"]
# host-only instrumentation: every sanitizer flag applies to the host pass
SAN_FLAGS = ["-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _compile(src: str, verbose: bool, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_BUILD if sanitize else BUILD, os.path.basename(src) + ".o")
    flags = FLAGS + SAN_FLAGS if sanitize else FLAGS
    cmd = [HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link the library; returns its path.  With
    `sanitize` the library is librpot_san.so; its sanitizer symbols resolve
    from the runtime preloaded at run time (sanitizer_env())."""
    out = SAN_LIB if sanitize else LIB
    os.makedirs(SAN_BUILD if sanitize else BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sanitize), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def sanitizer_env(env=None) -> dict:
    """Environment for a child process that loads librpot_san.so: the
    AddressSanitizer runtime (which carries the UndefinedBehaviorSanitizer
    handlers) put first in LD_PRELOAD, leak checks off (the interpreter itself
    is not instrumented), abort on the first report."""
    env = dict(os.environ if env is None else env)
    rt = subprocess.check_output([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        raise FileNotFoundError("AddressSanitizer runtime not found next to hipcc's clang")
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = rt + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["RPOT_LIB"] = SAN_LIB
    return env


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
