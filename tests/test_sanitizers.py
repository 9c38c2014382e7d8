"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- the oracle's C part, built with gcc's sanitizers, runs every oracle pin;
- the library's host-only sources (C ABI, index files, batching, serving, memory),
  built with clang's sanitizers and linked with the plain kernel objects, run the CPU
  ABI tests: argument checks and the corrupted index files of the loader.

Each runs in a child process with its sanitizer runtime preloaded; any report (memory
error or undefined behaviour) aborts the child and fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_BASE = {"ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
            "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(env_extra, args):
    env = dict(os.environ)
    env.update(ENV_BASE)
    env.update(env_extra)
    r = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    return out


def test_oracle_under_asan_and_ubsan():
    from oracle import oracle as O
    O.build(sanitize=True)
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(libasan)
    out = _run({"LD_PRELOAD": libasan, "RKMIPS_ORACLE_SANITIZE": "1"},
               ["-c", "import sys, ctypes; from oracle import oracle as O; "
                      "assert O._L()._name.endswith('liborc_san.so'); "
                      "assert hasattr(ctypes.CDLL(None), '__asan_init'); "
                      "import pytest; sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', "
                      "'tests/test_oracle_pins.py']))"])
    assert "passed" in out and "failed" not in out


def test_host_library_under_asan_and_ubsan():
    from paper_2211_12751_amd import build as B
    lib = B.build_sanitized()
    rt = B.asan_runtime()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("the clang AddressSanitizer runtime is not installed")
    out = _run({"LD_PRELOAD": rt, "RKMIPS_LIB": lib},
               ["-c", "import sys, ctypes; from paper_2211_12751_amd import rkmips as R; "
                      "assert R.LIB_PATH.endswith('librkmips_san.so'); "
                      "assert hasattr(ctypes.CDLL(None), '__asan_init'); "
                      "import pytest; sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', "
                      "'tests/test_abi_cpu.py']))"])
    assert "passed" in out and "failed" not in out
