"""Build the gfx950 shared library libncl_kkt.so in-tree.

Host analysis sources (.cpp) are compiled with g++, the HIP sources with
hipcc for gfx950, and everything is linked by hipcc into
paper_2510_05885_amd/libncl_kkt.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libncl_kkt.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for f in sorted(os.listdir(SRC)):
        src = os.path.join(SRC, f)
        obj = os.path.join(BUILD, f + ".o")
        if f.endswith(".cpp"):
            cmd = ["g++"] + CXX_FLAGS + ["-I", SRC, "-c", src, "-o", obj]
        elif f.endswith(".hip"):
            cmd = [HIPCC] + HIP_FLAGS + ["-I", SRC, "-c", src, "-o", obj]
        else:
            continue
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
