"""Build libffp.so (HIP for gfx950) in-tree with hipcc.

python -m paper_2101_11408_amd.build      # or build() from Python
"""

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN = os.path.join(PKG, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libffp.so")
ARCH = os.environ.get("FFP_OFFLOAD_ARCH", "gfx950")

SOURCES = ["ffp_kernels.hip", "ffp_capi.cpp", "ffp_server.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-pthread",
    "-Wno-unused-function",
    "-Wno-unknown-warning-option",
    # keep the compiler from emitting packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(GEN, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_table.py"),
                           os.path.join(GEN, "ffp_table.inc")])
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", GEN,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    build_strtod_ctx()
    return LIB


STRTOD_LIB = os.path.join(LIBDIR, "libstrtod_ctx.so")


def build_strtod_ctx() -> str:
    """The C library's strtod / strtof timed over a buffer: a context line
    beside the GPU parser's measurements (plain C, host only)."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler for the strtod context library")
    tmp = STRTOD_LIB + ".tmp"
    subprocess.check_call([cc, "-O2", "-shared", "-fPIC", "-pthread",
                           os.path.join(CSRC, "strtod_ctx.c"), "-o", tmp])
    os.replace(tmp, STRTOD_LIB)
    return STRTOD_LIB


if __name__ == "__main__":
    print(build(verbose=True))
