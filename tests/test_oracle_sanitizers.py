"""The CPU oracle and the paper-design baseline under AddressSanitizer and
UndefinedBehaviorSanitizer (gcc): oracle/sanitize_main.c drives every
function over shapes from 1x1 to 40x41, radii 1-12 and extreme thresholds,
with exact-size buffers, so an out-of-bounds access, a leak or undefined
behaviour fails the run.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", f) for f in ("sanitize_main.c", "canny_oracle.c", "paper_design.c")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cc = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe] + SRC + ["-lm"]
    r = subprocess.run(cc, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("gcc without sanitizer runtimes: " + r.stderr[:200])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    if run.returncode != 0 and "does not come first in initial library list" in run.stderr:
        pytest.skip("a library preloaded into every process keeps ASan from starting first")
    assert run.returncode == 0, run.stderr[-4000:]
    assert "sanitized oracle run: ok" in run.stdout
