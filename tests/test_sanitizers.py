"""The FP64 oracle and the host code of libpanda.so under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.  Each part's CPU tests run in a
subprocess with the sanitizer runtime preloaded (gcc's for the oracle, the
ROCm clang's for the library, whose host code hipcc built with -Xarch_host
sanitizers); a sanitizer report, or any failure, fails the test.  The
sanitized libraries are built by __graft_entry__.build()."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def run_under(runtime, env_flag, files):
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", **{env_flag: "1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider"] + files,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_under_asan_ubsan():
    from oracle import oracle as O
    O.build(force=False, sanitize=True)
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    files = [os.path.join("tests", f) for f in ("test_oracle_pins.py", "test_pearson_pins.py",
                                                 "test_null_pins.py", "test_warmstart_pins.py")]
    out = run_under(rt, "ORACLE_SANITIZED", files)
    assert " passed" in out


def test_library_host_code_under_asan_ubsan():
    lib = os.path.join(ROOT, "paper_1507_07039_amd", "libpanda_san.so")
    if not os.path.exists(lib):
        pytest.skip("libpanda_san.so not built (__graft_entry__.build() builds it)")
    rts = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("the ROCm clang AddressSanitizer runtime is not installed")
    out = run_under(rts[0], "PANDA_LIB_SANITIZED", [os.path.join("tests", "test_abi.py")])
    assert " passed" in out
