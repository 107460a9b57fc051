"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): oracle/sanitize_driver.c calls every entry point of
oracle/lbm_oracle.c on small inputs (both collision forms, scalar and tensor
permeability, walls, a force field, local K_eff runs, a NaN state, block
averages), with OpenMP on; any sanitizer finding aborts the run."""
import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "sanitize_driver"
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
           os.path.join(ORACLE, "sanitize_driver.c"), os.path.join(ORACLE, "lbm_oracle.c"),
           "-lm", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("no AddressSanitizer runtime for gcc here: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize_driver ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
