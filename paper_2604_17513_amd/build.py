"""Builds the HIP library libflash_mi355x.so in-tree for gfx950 (hipcc)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflash_mi355x.so")
OBJ = os.path.join(HERE, "_build")

COMMON = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# per-source extra flags: the contact predicate is evaluated without FMA contraction
SOURCES = {
    "flash_detect.hip": ["-ffp-contract=off"],
    "flash_kernels.hip": [],
    "flash_host.hip": [],
    "flash_state.hip": [],
    "flash_lite.hip": [],
    "flash_render.hip": [],
    "flash_mlp.hip": [],
    "flash_mlp_host.hip": [],
}


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for src, extra in SOURCES.items():
        obj = os.path.join(OBJ, src.replace(".hip", ".o"))
        jobs.append(([hipcc, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj], obj))

    def compile_one(job):
        if verbose:
            print(" ".join(job[0]), flush=True)
        subprocess.run(job[0], check=True)
        return job[1]

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, jobs))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
