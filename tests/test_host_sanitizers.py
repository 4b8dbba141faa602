"""The host side of the library under AddressSanitizer and UndefinedBehavior-
Sanitizer: the library is rebuilt with both sanitizers on its host code only
(device code is compiled as usual), and the CPU tests that call into it (ABI
exports and argument validation, the shearlet filter taps, the workload
generators) run again in a child process with the instrumented build loaded
through OKRIG_LIB. Any sanitizer report fails the test."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]
CPU_TESTS = ["tests/test_abi_cpu.py", "tests/test_edge_filters_cpu.py", "tests/test_workloads.py"]


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2303_09523_amd import build as B
    runtime = _asan_runtime()
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc is not available")
    if runtime is None:
        pytest.skip("the clang AddressSanitizer runtime is not available")
    objdir = tmp_path / "obj"
    objdir.mkdir()

    def compile_one(src):
        obj = str(objdir / (os.path.splitext(src)[0] + ".o"))
        cmd = [B.hipcc(), *B.FLAGS, *HOST_SAN, "-c", os.path.join(B.CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = str(tmp_path / "libokrig_san.so")
    res = subprocess.run([B.hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}",
                          "-shared-libasan", "-Xarch_host", "-fsanitize=address",
                          "-Xarch_host", "-fsanitize=undefined", *objs, "-o", lib],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]

    env = dict(os.environ)
    env.update({
        "OKRIG_LIB": lib,
        "LD_PRELOAD": runtime,
        # the interpreter and its extension modules are not instrumented: no
        # leak report for them, and allocations may cross runtimes
        "ASAN_OPTIONS": "detect_leaks=0:alloc_dealloc_mismatch=0:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          "-m", "not gpu", *CPU_TESTS], cwd=ROOT, env=env,
                         capture_output=True, text=True, timeout=600)
    out = run.stdout + run.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert run.returncode == 0, out[-4000:]
