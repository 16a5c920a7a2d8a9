"""The library's host code (dg_host.cpp: configuration checks, tables, the driving update, the
MLP shape helpers, argument validation) under AddressSanitizer and UndefinedBehaviorSanitizer, on
the CPU: dg_host.cpp is rebuilt instrumented (host pass only; the device code and the other objects
are the normal build), linked into a copy of the library in a temporary directory, and the host ABI
tests run against it in a child process (DGMI_LIB) with clang's ASan runtime preloaded.  Leak
detection is off: the interpreter's own allocations outlive it by design."""
import os
import subprocess
import sys

import pytest

from paper_1602_09079_amd import build as pb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def _asan_runtime():
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if os.path.isabs(path) and os.path.exists(path):
        return path
    base = "/opt/rocm/lib/llvm/lib/clang"
    for ver in sorted(os.listdir(base)) if os.path.isdir(base) else []:
        for sub in ("lib/linux/libclang_rt.asan-x86_64.so", "lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"):
            p = os.path.join(base, ver, sub)
            if os.path.exists(p):
                return p
    return None


@pytest.mark.slow
def test_host_abi_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    objs = [os.path.join(pb.HERE, "_build", s + ".o") for s in pb.SOURCES if s != "dg_host.cpp"]
    if rt is None or not os.path.exists(HIPCC) or not all(os.path.exists(o) for o in objs):
        pytest.skip("no clang ASan runtime, hipcc or normal build objects")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-shared-libasan"]
    host_o = str(tmp_path / "dg_host_san.o")
    lib = str(tmp_path / "libdgmi_san.so")
    flags = [f for f in pb.HIP_FLAGS if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer"]
    subprocess.check_call([HIPCC] + flags + san + ["-I", os.path.join(ROOT, "include"), "-I", pb.CSRC, "-x", "hip",
                                                   "-c", os.path.join(pb.CSRC, "dg_host.cpp"), "-o", host_o])
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + san + ["-o", lib] + objs +
                          [host_o, "-lhipfft"])
    env = dict(os.environ)
    env.update(DGMI_LIB=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the child loads the instrumented build
    probe = ("from paper_1602_09079_amd import dg\n"
             "dg.lib()\n"
             "print(sum('libdgmi_san.so' in l for l in open('/proc/self/maps')) > 0)\n")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().splitlines()[-1] == "True", r.stdout[-1000:] + r.stderr[-2000:]
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
           os.path.join(ROOT, "tests", "test_abi_host.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = r.stdout[-2000:] + "\n" + r.stderr[:3000]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
