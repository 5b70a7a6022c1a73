"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer: the C oracle is
rebuilt with both (undefined behaviour fatal) and the whole pin suite runs against it in a
child process with the sanitizer runtimes preloaded.  A planted out-of-bounds write (an
output buffer one element short) must be caught, which shows the instrumentation is live."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    return p.stdout.strip() if p.returncode == 0 and os.path.isabs(p.stdout.strip()) else None


@pytest.fixture(scope="module")
def san_env():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan and os.path.exists(asan) and os.path.exists(ubsan)):
        pytest.skip("gcc sanitizer runtimes not installed")
    path = oracle.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=f"{asan} {ubsan}", ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", RANPHY_REF_LIB=path)
    return env


def test_pins_pass_under_sanitizers(san_env):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=san_env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr


def test_planted_overflow_is_caught(san_env):
    code = (
        "import ctypes, numpy as np, oracle\n"
        "L = oracle.lib()\n"
        "assert L._name.endswith('libranphy_ref_san.so'), L._name\n"
        "x = np.ones(64, np.complex128); nv = np.ones(64, np.float64)\n"
        "out = np.zeros(64 * 4 - 1, np.float64)  # one LLR short\n"
        "L.ranphy_ref_llr_batch(64, 4, x.ctypes.data, nv.ctypes.data, out.ctypes.data)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=san_env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr and "WRITE" in r.stderr, \
        r.stderr[-2000:]
