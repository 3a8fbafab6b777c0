"""Build the in-tree HIP library libstmg.so for gfx950 (hipcc, no JIT cache)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstmg.so")
SOURCES = ["host.cpp", "kernels.hip", "learned.hip", "stmg_api.hip"]
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
    "--offload-arch=gfx950",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose=True):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(SRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc] + FLAGS + ["-c", os.path.join(SRC, src), "-o", obj]
        cmd.remove("-shared")
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # the sources compile independently: run them side by side
    procs = [subprocess.Popen(c) for c in cmds]
    codes = [p.wait() for p in procs]
    for c, rc in zip(cmds, codes):
        if rc != 0:
            raise subprocess.CalledProcessError(rc, c)
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + objs + ["-o", tmp, "-Wl,-rpath,/opt/rocm/lib:/opt/rocm/llvm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
