"""Build the HIP library libmpm_mag.so for gfx950 (in-tree, next to this file).

The engine is compiled once per (precision, dimension) variant in parallel, then
linked with the C-ABI translation unit and the design front end. All device code is built with packed
FP32 instructions disabled and hardware floating-point atomics enabled.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmpm_mag.so")
ARCH = os.environ.get("MPM_OFFLOAD_ARCH", "gfx950")

COMMON = ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}"]

VARIANTS = [("float", 2, "make_engine_f2"), ("float", 3, "make_engine_f3"),
            ("double", 2, "make_engine_d2"), ("double", 3, "make_engine_d3")]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    for real, dim, fac in VARIANTS:
        obj = os.path.join(BUILD, f"engine_{real[0]}{dim}.o")
        jobs.append([hipcc] + COMMON + [f"-DMPM_REAL={real}", f"-DMPM_DIM={dim}", f"-DMPM_FACTORY={fac}",
                                        "-c", os.path.join(CSRC, "engine_inst.hip"), "-o", obj])
    jobs.append([hipcc] + COMMON + ["-c", os.path.join(CSRC, "abi.hip"), "-o", os.path.join(BUILD, "abi.o")])
    jobs.append([hipcc] + COMMON + ["-c", os.path.join(CSRC, "design.hip"), "-o", os.path.join(BUILD, "design.o")])
    with cf.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        for cmd in jobs:
            if verbose:
                print(" ".join(cmd), flush=True)
        list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
