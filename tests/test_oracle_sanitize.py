"""The oracle's C source under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_driver.c runs every phase of the oracle's solver (Sinkhorn warm-up, eval,
sparsify, CG, Armijo trials, Algorithm 3 and the certificate, the outer update) and its plain
passes on small problems: FP64 and FP32 cost, rho = 0 (IBN), (E)IBSN, a single source and a
single target.  Built with gcc and run in a subprocess; any sanitizer report fails it.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_sanitize")
    src = [os.path.join(ROOT, "oracle", "ibsn_oracle.c"),
           os.path.join(ROOT, "oracle", "sanitize_driver.c")]
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", *src, "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok"), r.stdout
