"""Host logic of the library on the CPU, built with AddressSanitizer and
UndefinedBehaviorSanitizer from the library's own headers:

* pipeline_plan_driver.cpp: the software-pipeline schedule of
  fdfb_bootstrap_pipeline (csrc/pipeline_plan.h) over 3000 random job mixes
  (empty and one-sample jobs, 1 to 5 sign rotations per sample, narrow and
  wide geometries, resident capacities from 1 to 512, 1 to 8 rounds per
  launch).  Every job's sign accumulators are covered once, in job order, cut
  only at whole samples and work items; each job's ModSwitch precedes its first
  sign launch, its public mux follows its last, its function rotation comes in
  a later launch and its output right after it; no launch is empty, and every
  launch followed by more sign work holds its rounds of the capacity.
* arena_driver.cpp: the serving engine's first-fit arena (csrc/arena.h)
  against a shadow map of its block over random allocations and releases.
  Every allocation succeeds exactly when a free run fits, at the lowest such
  offset, no unit is handed out twice, the free ranges are always the maximal
  free runs, and releasing everything leaves one block."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2109_02731_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
@pytest.mark.parametrize("driver", ["pipeline_plan_driver.cpp", "arena_driver.cpp"])
def test_host_logic_invariants(driver):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "driver")
        base = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-I", CSRC, os.path.join(HERE, driver), "-o", exe]
        built = subprocess.run(base[:1] + ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"] + base[1:],
                               capture_output=True, text=True)
        if built.returncode != 0 and "asan" in built.stderr.lower():
            built = subprocess.run(base, capture_output=True, text=True)  # no sanitizer runtime here
        assert built.returncode == 0, built.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
        assert run.stdout.strip().endswith("ok")
