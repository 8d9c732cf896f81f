"""The boundary's host code (planning, validation, descriptors) under
AddressSanitizer and UndefinedBehaviorSanitizer: the CPU tests of the C-ABI
run in a child process against libsfd built with sanitized host code, the
sanitizer runtime preloaded (CPU only; no compute call is made)."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_abi_tests_pass_under_address_and_undefined_behaviour_sanitizers():
    from paper_1001_4309_amd import build as b

    rt = _asan_runtime()
    if rt is None:
        pytest.fail("the clang AddressSanitizer runtime is missing from /opt/rocm/lib/llvm")
    if not os.path.exists(b.SAN_LIB) or os.path.getmtime(b.SAN_LIB) < os.path.getmtime(b.LIB):
        b.build_sanitized()
    # The host code is instrumented (it calls into the sanitizer runtime).
    syms = subprocess.run(["nm", "-D", "--undefined-only", b.SAN_LIB], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    env = dict(os.environ, SFD_LIB_PATH=b.SAN_LIB, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = ("import sys, pytest, paper_1001_4309_amd._lib as L; "
            "assert L.LIB_PATH.endswith('libsfd_san.so'), L.LIB_PATH; "
            "sys.exit(pytest.main(['tests/test_abi_cpu.py', '-x', '-q', '-p', 'no:cacheprovider']))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-4000:] + r.stderr[-4000:])
    assert " passed" in r.stdout
