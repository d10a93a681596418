"""The oracle's C source under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): key generation and a full-domain bootstrap of every message at
n=64 N=256 t=8 must run without a report and decrypt correctly."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_san")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", os.path.join(HERE, "oracle_sanitize_driver.c"), "-lm", "-o", exe]
        built = subprocess.run(cmd, capture_output=True, text=True)
        if built.returncode != 0 and "asan" in built.stderr.lower():
            pytest.skip("sanitizer runtime not available: " + built.stderr[-200:])
        assert built.returncode == 0, built.stderr[-2000:]
        # link-order check off: the environment may preload a library ahead of the ASan runtime
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
        assert run.stdout.strip().endswith("ok")
        assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
