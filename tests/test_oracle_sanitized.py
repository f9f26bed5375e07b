"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's own tests (tests/test_oracle.py: pins against closed forms, brute force
and the literal/fast-mode agreement, on every fixture they use) run in a child process
that loads the sanitized build of oracle/dpcg_oracle.c (-fsanitize=address,undefined,
UB fatal) with the ASan runtime preloaded.  Any out-of-bounds access, use after free or
undefined operation in the oracle fails this test.  CPU only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def san_env():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's ASan runtime is not installed")
    sys.path.insert(0, ROOT)
    from oracle.build import build
    build(sanitize=True)
    env = dict(os.environ)
    env.update(ORACLE_SANITIZED="1", LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONDONTWRITEBYTECODE="1")
    return env


def test_sanitized_build_is_the_one_loaded(san_env):
    probe = ("import ctypes, oracle; oracle.lib(); "
             "maps = open('/proc/self/maps').read(); "
             "assert 'liboracle_san.so' in maps and 'liboracle.so' not in maps, 'wrong oracle library'; "
             "ctypes.CDLL(None).__asan_init; print('ok')")
    p = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=san_env, capture_output=True, text=True,
                       timeout=300)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout + p.stderr


def test_oracle_tests_pass_under_asan_and_ubsan(san_env):
    p = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle.py", "-q", "-x", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=san_env, capture_output=True, text=True, timeout=1200)
    out = p.stdout + p.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]
