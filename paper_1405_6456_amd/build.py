"""Builds libalofdft.so (HIP, gfx950) in-tree with hipcc.

The stencil instantiations for each radius 1..8 are compiled as separate
translation units in parallel, then linked with the engine into one library.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libalofdft.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions in any kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
RADII = range(1, 9)


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def jobs():
    out = [([hipcc(), *FLAGS, "-c", os.path.join(CSRC, "engine.hip"), "-o", os.path.join(OBJ, "engine.o")],
            "engine")]
    for r in RADII:
        out.append(([hipcc(), *FLAGS, f"-DALOFDFT_RADIUS={r}", "-c", os.path.join(CSRC, "stencil_inst.hip"),
                     "-o", os.path.join(OBJ, f"stencil_r{r}.o")], f"stencil r={r}"))
    return out


def build(verbose=True, workers=None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    todo = jobs()
    workers = workers or min(len(todo), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))

    def run(job):
        cmd, name = job
        res = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
        return name, res.returncode, err

    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(run, todo))
    failed = False
    for name, rc, err in results:
        if err.strip() and verbose:
            print(f"[{name}]\n{err}", flush=True)
        failed |= rc != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    objs = [os.path.join(OBJ, "engine.o")] + [os.path.join(OBJ, f"stencil_r{r}.o") for r in RADII]
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
