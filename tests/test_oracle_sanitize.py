"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer, CPU only:
tests/oracle_sanitize_driver.c runs every entry point on small grids of every
model and option (limiters, characteristic variables, TENO6-A, THINC, sixth-order
viscous fluxes, viscosity laws, mixed boundary conditions, lines and single
cells) and must finish with no sanitizer report."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitize")
        flags = ["-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
                 "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
        subprocess.run(["gcc", *flags, os.path.join(HERE, "oracle_sanitize_driver.c"), "-o", exe, "-lm"],
                       check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        print(r.stdout[-2000:], r.stderr[-4000:])
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runs, 0 non-finite" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
