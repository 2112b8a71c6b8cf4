"""Build libnfm.so (HIP for gfx950) in-tree with hipcc.

Every HIP source is compiled with packed-FP32 instructions disabled and without
floating-point contraction (the FP64 table and recursion arithmetic follows the
operation order written in the source)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libnfm.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["api.cpp", "mlp_api.cpp", "stats.cpp", "lattice.hip", "tables.hip", "sweep.hip", "recursion.hip", "wl.hip", "features.hip",
           "mlp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
         # private arrays stay in registers or scratch, never in LDS: the sweep kernel owns
         # its whole LDS allocation (checked at launch)
         "-mllvm", "-disable-promote-alloca-to-lds"]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (a checking build of the library's
# host code for the CPU test suite; the GPU code is compiled as usual). Each -fsanitize= applies
# to the host compilation only.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + (".san.o" if sanitize else ".o"))
    lang = ["-x", "hip"]
    cmd = [HIPCC, *lang, *FLAGS, *(SANITIZE if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr[-4000:]}")
    return obj


def build(verbose: bool = True, sanitize: bool = False) -> str:
    """Compile every source and link libnfm.so. sanitize=True links the host code against the
    address and undefined-behaviour sanitizers (run Python with the clang ASan runtime preloaded,
    e.g. LD_PRELOAD=$(hipcc -print-file-name=libclang_rt.asan-x86_64.so) ASAN_OPTIONS=detect_leaks=0);
    build again without it afterwards."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = OUT + ".tmp"
    # -z defs: an undefined symbol is a link error here, not a load error on the GPU host (the
    # sanitized build takes the sanitizer runtimes from the preloading process instead)
    link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libasan"] \
        if sanitize else ["-Wl,-z,defs"]
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *link, *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
