"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host only).

`tests/oracle_sanitize_main.c` calls every oracle entry point (whole solves of several
sizes, subsets and leading dimensions, argument errors, a B that is not positive
definite, the stages on their own and the forced QL failure); it is compiled with the
oracle source by gcc with -fsanitize=address,undefined and no recovery, and run.  An
out-of-bounds access, use after free, leak or undefined operation in the oracle ends the
run with a non-zero status.  (OpenMP is left out of this build: its pragmas only split
independent loops.)
"""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_address_and_undefined_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitized")
        cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-Wno-unknown-pragmas",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               os.path.join(ROOT, "oracle", "hgv_oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c"),
               "-o", exe, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and ("asan" in r.stderr.lower() or "ubsan" in r.stderr.lower()):
            pytest.skip("sanitizer runtimes not available: " + r.stderr[-300:])
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert run.returncode == 0, (run.stdout[-1000:], run.stderr[-3000:])
        assert "all checks passed" in run.stdout
