"""Build libgpgomea_eval.so (HIP for gfx950) in the package directory.

    python paper_2605_30954_amd/build.py [--jobs N] [--save-temps]

(run by path: importing the package would load the library being rebuilt)

Every translation unit under csrc/ is compiled by hipcc in parallel and
linked into one shared library; the build always recompiles.
"""
import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgpgomea_eval.so")
BUILD = os.path.join(PKG, "_build")
ARCH = "gfx950"

SOURCES = ["codec.cpp", "api.cpp", "k_prep.hip", "k_forward.hip", "k_adjoint.hip", "k_opcost.hip", "k_constopt.hip", "k_designs.hip"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
            "-Wall", "-Wno-unused-function",
            # never emit packed FP32 math (v_pk_add/mul/fma_f32)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # the interpreters branch on wave-uniform values only: leave uniform
            # regions unstructurized (plain scalar branches, fewer flow blocks and
            # fewer register copies at the joins)
            "-mllvm", "-structurizecfg-skip-uniform-regions=true"]


def compile_one(src, save_temps=False):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + common_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if save_temps:
        cmd += ["--save-temps"]
    r = subprocess.run(cmd, cwd=BUILD, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    return obj, err


def build(jobs=None, save_temps=False, verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: compile_one(s, save_temps), SOURCES))
    for (obj, err) in results:
        if err.strip() and verbose:
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--save-temps", action="store_true")
    a = ap.parse_args()
    build(a.jobs, a.save_temps)
