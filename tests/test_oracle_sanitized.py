"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle source is compiled with -fsanitize=address,undefined (host code
only, nothing here touches a GPU) and the pin tests run against that build
in a child process that preloads the ASan runtime.  Any out-of-bounds access,
use after free or undefined operation in the oracle ends the child with an
error and fails this test.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_pins_pass_under_address_and_ub_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ)
    env["NNCP_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = asan
    # the interpreter's own allocations are not the oracle's: no leak report
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"),
           os.path.join(ROOT, "tests", "test_oracle_pins_nls.py"), "-k", "not catch"]
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail


def test_sanitized_build_reports_a_planted_overrun(tmp_path):
    """The harness above does catch memory errors: an oracle copy whose Gram
    writes one entry past the end of its output dies under ASan."""
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    src = oracle.source_text()
    old = "      G[a * R + b] = s;\n"
    assert src.count(old) == 1
    bad = oracle.build_variant(str(tmp_path / "liboracle_overrun.so"),
                               src.replace(old, "      G[a * R + b + 1] = s;\n"),
                               extra_flags=oracle.SANITIZE_FLAGS)
    env = dict(os.environ, NNCP_ORACLE_LIB=bad, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    code = "import numpy as np, oracle; oracle.gram(np.ones((5, 16)))"
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr
