"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, no OpenMP) and driven through every entry point on a small graph with
self-loops, repeated arcs, an isolated node, a hub, a ragged replicate count
and a replicate offset: no sanitizer report, and the driver's consistency
checks hold (tests/oracle_sanitize_main.c)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "oracle_san")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-ffp-contract=off", "-Wno-unknown-pragmas",
               os.path.join(ROOT, "oracle", "fsg_oracle.c"),
               os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-o", exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        env.pop("LD_PRELOAD", None)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "oracle sanitizer run ok" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
