"""Build libpic.so in-tree with hipcc for gfx950.

Usage: python paper_2208_02382_amd/build.py   (or __graft_entry__.build()).  Run it by path:
importing the package loads the library this script builds.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpic.so")
# host build of the device double-double / IGF arithmetic, for CPU unit tests only
HOSTCHECK = os.path.join(HERE, "libpic_hostcheck.so")
# the bench's reference measurement of LDS atomic throughput (not part of libpic.so)
PROBE = os.path.join(HERE, "libpic_probe.so")
SOURCES = ["particles.hip", "sort.hip", "igf.hip", "fft.hip", "adjoint.hip", "noalloc.hip",
           "api.cpp"]

# -Xclang -target-feature -Xclang -packed-fp32-ops: no packed FP32 instructions are emitted.
# -munsafe-fp-atomics: float atomic adds map to the hardware global_atomic_add_f32/f64.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-function"]


# the double-double arithmetic of the integrated Green's function needs every + and - rounded
# on its own: no contraction of a*b + c into fma in that translation unit
PER_FILE = {"igf.hip": ["-ffp-contract=off"]}


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc] + FLAGS + PER_FILE.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc] + [f for f in FLAGS if not f.startswith("--offload")] + [
                "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
        if verbose and (r.stderr.strip()):
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    tmp = HOSTCHECK + ".tmp"
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           os.path.join(CSRC, "hostcheck.cpp"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hostcheck build failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, HOSTCHECK)
    tmp = PROBE + ".tmp"
    cmd = [hipcc] + FLAGS + ["-shared", os.path.join(CSRC, "probe_lds.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("probe build failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, PROBE)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
