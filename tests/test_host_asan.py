"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer, on the CPU.

ecg_solver.hip is compiled with the sanitizer on its host side only (the
device code is not instrumented) and linked with the kernels object of the
normal build and a small C++ driver (tests/host_asan_driver.cpp).  The
driver runs the argument validation of ecg_setup and, on valid input, the
domain-contiguous row permutation (the caller's order within a domain, and
the Morton key order with the keys from ecg_grid_morton_keys); both run
before the first device call, so without a GPU setup then reports
ECG_EDEVICE.  A
planted heap overflow, built the same way, must be reported, so that a
clean run means something."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1804_10629_amd", "csrc")
KOBJ = os.path.join(ROOT, "paper_1804_10629_amd", "_build", "libecg", "ecg_kernels.o")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-O1", "-g",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-sanitize-recover=undefined",
         "-Xarch_host", "-fno-omit-frame-pointer",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _tools():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    if not os.path.exists(KOBJ):
        pytest.skip("no kernels object: run the build first")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)


def _link(objs, out):
    r = _run([CLANG, *objs, "-fsanitize=address,undefined", "-L/opt/rocm/lib", "-lamdhip64",
              "-Wl,-rpath,/opt/rocm/lib", "-o", out])
    assert r.returncode == 0, r.stderr[-2000:]


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    return env


def test_sanitizer_reports_a_planted_overflow(tmp_path):
    _tools()
    src = tmp_path / "planted.cpp"
    src.write_text("#include <cstdio>\nint main() { volatile int* p = new int[4]; p[4] = 1;"
                   " std::printf(\"%d\\n\", p[0]); return 0; }\n")
    obj = str(tmp_path / "planted.o")
    r = _run([HIPCC, *FLAGS, "-c", str(src), "-o", obj])
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "planted")
    _link([obj], exe)
    r = _run([exe], env=_env())
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


def test_setup_host_code_is_clean_under_asan(tmp_path):
    _tools()
    sobj = str(tmp_path / "solver.o")
    r = _run([HIPCC, *FLAGS, "-c", os.path.join(CSRC, "ecg_solver.hip"), "-o", sobj])
    assert r.returncode == 0, r.stderr[-2000:]
    dobj = str(tmp_path / "driver.o")
    r = _run([HIPCC, *FLAGS, "-c", os.path.join(ROOT, "tests", "host_asan_driver.cpp"),
              "-o", dobj])
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "driver")
    _link([dobj, sobj, KOBJ], exe)
    r = _run([exe], env=_env())
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout, r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
