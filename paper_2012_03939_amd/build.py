"""Build the gfx950 HIP library libshapetrace.so in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed FP32 vector
instructions disabled and hardware float atomics enabled, then linked into one
shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libshapetrace.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["st_build.hip", "st_render.hip", "st_backward.hip", "st_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def _compile(src: str, build_dir: str = BUILD, defines=(), extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj


OUT_SANITIZE = os.path.join(HERE, "libshapetrace_san.so")
# host code only (argument validation, tables, sequencing): the GPU code objects
# are built as usual
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, out: str = OUT, defines=(), sanitize: bool = False) -> str:
    """Compile and link; `defines` (NAME=VALUE) override compile-time tuning
    constants, `out` names the library (default: next to this file).
    sanitize: host code with AddressSanitizer and UndefinedBehaviorSanitizer, as
    libshapetrace_san.so (loaded when SHAPETRACE_SANITIZE=1, with clang's ASan
    runtime preloaded into the process)."""
    if sanitize and out == OUT:
        out = OUT_SANITIZE
    build_dir = BUILD if out == OUT else os.path.join(os.path.dirname(os.path.abspath(out)),
                                                      "_build_san" if sanitize else "_build")
    os.makedirs(build_dir, exist_ok=True)
    extra = SANITIZE_FLAGS if sanitize else []
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, defines, extra), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=OUT)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    ap.add_argument("--sanitize", action="store_true", help="host code with ASan + UBSan (libshapetrace_san.so)")
    a = ap.parse_args()
    build(verbose=True, out=a.out, defines=a.defines, sanitize=a.sanitize)
    sys.exit(0)
