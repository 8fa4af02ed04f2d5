"""The library's host code under the address and undefined-behaviour sanitizers (CPU only).

Every source of the library is compiled with the sanitizers on its host side (device code is
built as usual), linked with tests/host/host_checks.cpp into one executable, and run: the C ABI's
argument validation and the serving scheduler's first-fit pool allocator (against a byte-map
model) must pass with no sanitizer report.  No call made there reaches a device."""
import concurrent.futures
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_2501_10709_amd import build as BUILD

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _tools():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not (os.path.exists(hipcc) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ not available")
    return hipcc


@pytest.mark.timeout(600)
def test_host_code_under_sanitizers():
    hipcc = _tools()
    flags = [f for f in BUILD.HIPCC_FLAGS if f not in ("-O3", "-fPIC")]
    with tempfile.TemporaryDirectory() as tmp:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc, *flags, "-O1", "-g", *SAN_HOST, "-c", os.path.join(BUILD.CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, f"{src}:\n{r.stderr[-4000:]}"
            return obj

        with concurrent.futures.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(compile_one, BUILD.SOURCES))
        for obj in objs:  # the host side of every object is instrumented
            syms = subprocess.run(["nm", "-u", obj], capture_output=True, text=True).stdout
            assert "__asan_" in syms and "__ubsan_" in syms, obj
        main_obj = os.path.join(tmp, "host_checks.o")
        cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{BUILD.INCLUDE}",
               f"-I{BUILD.CSRC}", "-c", os.path.join(HOST, "host_checks.cpp"), "-o", main_obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        exe = os.path.join(tmp, "host_checks")
        cmd = [CLANG, "-fsanitize=address,undefined", main_obj, *objs, "-L/opt/rocm/lib", "-lamdhip64",
               "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        env.pop("HIP_VISIBLE_DEVICES", None)
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr[-6000:]
        assert "host checks passed" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
