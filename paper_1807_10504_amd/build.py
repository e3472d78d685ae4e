"""Build the HIP library ``libibproj.so`` in-tree for gfx950.

Device translation units (``csrc/*.hip``) are compiled with hipcc; the host
FP64 interface-geometry units (``csrc/*.cpp``) with g++ and no floating-point
contraction, so that the B-spline relocation is reproducible bit for bit.
Objects go to ``_build/`` at the repository root.

    python -m paper_1807_10504_amd.build
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libibproj.so")
OBJ = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-I" + os.path.join(ROOT, "include")]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
              "-Wall", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cmds, objs = [], []
    for f in sorted(os.listdir(SRC)):
        src = os.path.join(SRC, f)
        if f.endswith(".hip"):
            o = os.path.join(OBJ, f[:-4] + ".o")
            cmds.append([HIPCC] + HIP_FLAGS + ["-c", src, "-o", o])
        elif f.endswith(".cpp"):
            o = os.path.join(OBJ, f[:-4] + ".o")
            cmds.append([CXX] + HOST_FLAGS + ["-c", src, "-o", o])
        else:
            continue
        objs.append(o)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    # the host units use OpenMP (GCC's runtime)
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
