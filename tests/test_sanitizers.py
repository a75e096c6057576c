"""Host C code under AddressSanitizer and UndefinedBehaviorSanitizer: the
FP64 oracle and the input generator, built with gcc and driven by
tests/sanitize_driver.c (edge sub-boxes, taps across the detector border,
a view that misses the volume, invalid arguments), which also checks that
box, point and full evaluations agree bit for bit and that the adjoint
identity holds.  Any sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_and_generator_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "tests", "sanitize_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "synth", "synth.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # (the ASan runtime need not come first among preloaded libraries)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(res.stdout, res.stderr)
    assert res.returncode == 0, res.stderr
    assert "all checks passed" in res.stdout
