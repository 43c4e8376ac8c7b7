"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
a copy of the oracle package is built with both in a temporary directory and
driven by oracle_sanitized_run.py in a child process (the sanitizer runtimes
are preloaded there), over seeded random graphs and the error paths.  Skipped
where gcc has no sanitizer runtimes."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _runtime(name):
    try:
        p = subprocess.check_output(["gcc", "-print-file-name=" + name], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not found")
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "mlp_oracle.py", "truss_oracle.c"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-std=c11", "-Wall",
                           "-Werror", "-o", str(pkg / "_truss_oracle.so"), str(pkg / "truss_oracle.c")])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan + ":" + ubsan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, os.path.join(HERE, "oracle_sanitized_run.py"), str(tmp_path), "120"],
                       env=env, cwd=str(tmp_path), capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok: 120 graphs" in r.stdout
