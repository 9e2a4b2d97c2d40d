"""Memory and undefined-behaviour checks of the host code on the CPU.

The oracle's C code is built with gcc's AddressSanitizer and
UndefinedBehaviorSanitizer (no recovery: the first report aborts) and the
oracle tests run against that build; the C ABI library is built with the
same sanitizers on its host code only (device code unchanged) and the ABI
tests, which exercise every host-side path (plan sizes and layout,
configuration checks, argument rejection before any device call), run
against it.  Each runs in a subprocess with the matching sanitizer runtime
preloaded, since the instrumented library is loaded into Python."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
           "OMP_NUM_THREADS": "2"}


def _run(tests, env, tmp_path):
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           "--rootdir", ROOT] + [os.path.join(ROOT, "tests", t) for t in tests]
    r = subprocess.run(cmd, cwd=str(tmp_path), env=dict(os.environ, **SAN_ENV, **env), capture_output=True,
                       text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    for bad in ("AddressSanitizer", "runtime error:", "LeakSanitizer"):
        assert bad not in out, out
    return out


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime not available")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-o", str(lib), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"],
                   check=True)
    out = _run(["test_oracle_projection.py", "test_oracle_render.py", "test_oracle_grad.py",
                "test_oracle_alpha_depth.py", "test_oracle_sh.py"],
               {"ORACLE_LIB": str(lib), "LD_PRELOAD": asan}, tmp_path)
    assert " passed" in out


def test_c_abi_host_code_under_address_and_ub_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    rt = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        res = subprocess.run([hipcc, "-print-resource-dir"], capture_output=True, text=True).stdout.strip()
        rt = os.path.join(res, "lib", "linux", "libclang_rt.asan-x86_64.so")
    if not os.path.exists(rt):
        pytest.skip("clang's AddressSanitizer runtime not available")
    lib = tmp_path / "librtg_san.so"
    # host code instrumented, device code as in the product build
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-o", str(lib), os.path.join(ROOT, "paper_2404_19706_amd", "csrc", "api.hip")], check=True,
                   capture_output=True)
    out = _run(["test_abi.py"], {"RTG_LIB": str(lib), "LD_PRELOAD": rt}, tmp_path)
    assert " passed" in out
