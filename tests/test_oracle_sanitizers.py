"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host/oracle_san_main.c calls every entry point of oracle/mqh_oracle.c
(assembly, products stored and entry by entry with and without row scaling,
sampled products, Golub-Kahan with and without reorthogonalisation including
a full-space breakdown, projected and dense Jacobi SVDs, lift, evaluation)
on small seeded inputs; it is built with gcc -fsanitize=address,undefined
and run as a child process, and any sanitizer report fails the test.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(ROOT, "oracle", "mqh_oracle.c"), os.path.join(HERE, "host", "oracle_san_main.c")]
OUT = os.path.join(ROOT, "_build", "oracle_san")


def test_oracle_under_asan_ubsan():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-o", OUT, *SRC, "-lm"]
    try:
        subprocess.run(cmd, check=True, capture_output=True, text=True)
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"sanitizer build unavailable: {e}")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    res = subprocess.run([OUT], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr, res.stderr
    assert res.stdout.count("steps kept") == 5
