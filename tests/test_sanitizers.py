"""The CPU suite under AddressSanitizer and UndefinedBehaviorSanitizer.

Two builds made for the test: the oracle (oracle/*.c, gcc) and the library's host code
(csrc/*.hip with host-only sanitizer flags; the device code as usual).  Each runs in a child
process with its sanitizer runtime preloaded: the oracle build under every CPU test that
loads the oracle, the library build under the host-side checks of the C ABI (argument
validation, plans, workspace sizes, the GEMM launch checks).  A sanitizer report makes the
child fail: ASan aborts on the first error and undefined behaviour is not recovered from.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, args):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    import oracle as O
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan):
        pytest.skip("gcc's libasan is not installed")
    lib = O.build_sanitized(str(tmp_path))
    out = _run({"LD_PRELOAD": libasan, "ORC_LIBRARY": lib},
               ["tests", "-m", "not gpu", "--ignore=tests/test_abi_host.py",
                "--ignore=tests/test_sanitizers.py"])
    assert " passed" in out


def test_library_host_code_under_sanitizers(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's ASan runtime is not installed")
    from paper_2607_24234_amd import build
    lib = build.build(out=str(tmp_path / "libqs_san.so"), objdir=str(tmp_path / "obj"), sanitize=True)
    out = _run({"LD_PRELOAD": rt[-1], "QS_LIBRARY": lib}, ["tests/test_abi_host.py"])
    assert " passed" in out
