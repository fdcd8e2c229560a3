"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehavior Sanitizer (CPU only): every oracle entry point on a small
synthetic scene (oracle/selftest.c, built with gcc), and the host side of the
C ABI -- argument checks, defaults, null handling -- built with its host code
instrumented (paper_1905_06700_amd/build.py, build_sanitized)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(cmd, **kw):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=300, **kw)


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "selftest")
    b = _run(["gcc", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1",
              "-Wall", "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "selftest.c"),
              os.path.join(ROOT, "oracle", "rt3d_oracle.c"), "-lm", "-o", exe])
    assert b.returncode == 0, b.stderr
    r = _run([exe])
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    from paper_1905_06700_amd import build
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc missing")
    exe = build.build_sanitized(str(tmp_path / "san"))
    r = _run([exe])
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "host_selftest: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
