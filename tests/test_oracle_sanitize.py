"""The oracle's C sweep built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, CPU only) and run through a driver that exercises every entry point of
oracle/sweep.c: per-line integer shifts of both signs and beyond the line length,
an output selection, every storage tier, the transpose and the rounding of
special values.  The driver's checks are fixed by the method (section II-A: an
integer shift is a permutation, the alpha = 1/2 tables from hand-derived
fractions conserve mass, the transpose satisfies the dot-product identity)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_sweep_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wall", "-Wno-unknown-pragmas",
           "-o", exe, os.path.join(HERE, "oracle_sanitize_main.c"),
           os.path.join(ROOT, "oracle", "sweep.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "unrecognized" in r.stderr:
        pytest.skip("gcc without sanitizer support")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe, os.path.join(HERE, "golden", "ab_k2_alpha_half.txt")],
                         capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr, run.stderr
    assert "all checks passed" in run.stdout
