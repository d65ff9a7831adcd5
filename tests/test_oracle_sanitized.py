"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle test-suite runs in a child process against an instrumented build
(host code only), so an out-of-bounds access, a use after free, a signed
overflow or a misaligned access anywhere the tests reach fails here."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _libasan():
    gcc = shutil.which("gcc")
    if gcc is None:
        return None
    path = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_suite_clean_under_asan_and_ubsan():
    asan = _libasan()
    if asan is None:
        pytest.skip("gcc's libasan is not available")
    env = dict(os.environ, LBM_ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_numbering.py", "test_oracle_trt.py", "test_oracle_adjoint.py",
              "test_oracle_storage.py")]
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in res.stderr, tail
    assert os.path.exists(os.path.join(ROOT, "oracle", "_liblbm_oracle_san.so"))
