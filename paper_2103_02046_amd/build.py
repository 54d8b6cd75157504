"""Compile libp3m.so for gfx950 with hipcc (in-tree, no JIT).

    python -m paper_2103_02046_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libp3m.so")
SOURCES = ["api.hip", "placement.hip", "sort.hip", "pp.hip", "mesh.hip", "fft.hip", "lattice.hip", "diag.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # no packed FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    for s in SOURCES:
        obj = os.path.join(SRC, os.path.splitext(s)[0] + ".o")
        cmd = [hipcc] + [f for f in FLAGS if f != "-shared"] + ["-c", os.path.join(SRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE)))
        objs.append(obj)
    failed = []
    for s, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            failed.append((s, err.decode()))
        elif verbose and err:
            sys.stderr.write(err.decode())
    if failed:
        for s, e in failed:
            sys.stderr.write(f"---- {s}\n{e}\n")
        raise RuntimeError("hipcc failed on " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
