"""The library's host code under AddressSanitizer, on the CPU.

The library's sources are compiled for the host only (no device code) with ASan and linked
against tests/hoststub/hip_stub.cpp, a stand-in HIP runtime in which device memory is host
memory, kernel launches do nothing, and streams, events and graphs are tracked objects: using or
destroying a released handle, destroying a graph executable whose launch may still run,
synchronising a capturing stream or ending a capture with a forked stream unjoined aborts the
run.  tests/hoststub/lifetimes.cpp then drives the C ABI through the create / track / destroy
sequences of the GPU tests, among them two batches tracked one after the other with the first
batch and its beams torn down in between (the order of Python's rebinding), and teardowns right
after enqueued work with no synchronisation.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2208_02382_amd", "csrc")
STUB = os.path.join(ROOT, "tests", "hoststub")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_ASAN = ["-Xarch_host", "-fsanitize=address"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr[-4000:])
    return r


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ not installed")
    out = tmp_path_factory.mktemp("asan")
    common = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer"] + HOST_ASAN
    jobs = []
    for src in ("particles.hip", "sort.hip", "igf.hip", "fft.hip", "adjoint.hip"):
        jobs.append([HIPCC, "--offload-arch=gfx950", "--offload-host-only", "-Xclang",
                     "-target-feature", "-Xclang", "-packed-fp32-ops"] + common +
                    ["-c", os.path.join(CSRC, src), "-o", str(out / (src + ".o"))])
    jobs.append([HIPCC] + common + ["-c", os.path.join(CSRC, "api.cpp"), "-o", str(out / "api.o")])
    jobs.append([HIPCC] + common + ["-c", os.path.join(STUB, "hip_stub.cpp"),
                                    "-o", str(out / "stub.o")])
    jobs.append([HIPCC] + common + ["-I" + os.path.join(ROOT, "include"), "-c",
                                    os.path.join(STUB, "lifetimes.cpp"), "-o",
                                    str(out / "lifetimes.o")])
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for j in jobs]
    for j, p in zip(jobs, procs):
        o, e = p.communicate()
        assert p.returncode == 0, "%s\n%s" % (" ".join(j), e[-4000:])
    # the host objects reference the (absent) device code objects by name: give them storage
    objs = sorted(str(p) for p in out.glob("*.o"))
    nm = _run(["nm", "-u"] + objs).stdout
    names = sorted({w for w in nm.split() if w.startswith("__hip_fatbin_")})
    (out / "fatbin.cpp").write_text("".join('extern "C" { char %s[16]; }\n' % n for n in names))
    _run([CLANG, "-c", str(out / "fatbin.cpp"), "-o", str(out / "fatbin.o")])
    exe = out / "lifetimes"
    _run([CLANG, "-fsanitize=address", "-o", str(exe)] + objs + [str(out / "fatbin.o")])
    return exe


def test_host_paths_are_clean_under_asan(harness):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    r = subprocess.run([str(harness)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-6000:]
    assert "0 failures" in r.stdout and "0 leaked handles" in r.stdout, r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr
