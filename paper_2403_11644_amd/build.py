"""Build the HIP library libptd.so for gfx950 with hipcc (in-tree).

The host-only C++ sources (csrc/*.cpp) compile with the system C++ compiler
and link into the same library.

Run as ``python -m paper_2403_11644_amd.build``.  hipcc cross-compiles for
gfx950 without a GPU present.  Packed FP32 instructions are switched off
(``-packed-fp32-ops``) and FMA contraction is disabled so the butterfly
network is plain IEEE adds.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libptd.so")
ARCH = os.environ.get("PTD_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3",
    "--offload-arch=" + ARCH,
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-ffp-contract=off", "-Wall"]


def cxx() -> str:
    for cand in (os.environ.get("CXX"), shutil.which("g++"), "/usr/bin/g++"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("no host C++ compiler found (g++)")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libptd.so)")


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + sorted(glob.glob(os.path.join(CSRC, "*.cpp")))


def _jobs() -> int:
    env = os.environ.get("MAX_JOBS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, min(8, os.cpu_count() or 1))


def _filter(stderr: str) -> str:
    # the host pass warns that it does not know the packed-fp32 feature; drop that noise
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False) -> str:
    """Compile every csrc/*.hip into libptd.so; always recompiles.

    Translation units compile in parallel into a private object folder, then
    one link step writes the library.
    """
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = "-I" + os.path.join(ROOT, "include")
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + ".o")
        if src.endswith(".cpp"):
            cmd = [cxx()] + CXX_FLAGS + [inc, "-c", src, "-o", obj]
        else:
            cmd = [hipcc()] + compile_flags + [inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        err = _filter(res.stderr)
        if res.returncode != 0:
            raise RuntimeError("%s failed on %s:\n%s" % (os.path.basename(cmd[0]), os.path.basename(src), err))
        if verbose and err.strip():
            print(err, file=sys.stderr)
        return obj

    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(_jobs(), len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread"] + objs + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + _filter(res.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
