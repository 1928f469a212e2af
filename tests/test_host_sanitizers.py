"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host/capi_san is a build of every library source with host-side ASan
and UBSan (device code as usual) linked with tests/host/capi_san_main.cpp,
which drives the C ABI.  Without a GPU it runs the argument checks only (every
entry point rejects bad arguments before device work); the GPU test runs all
entry points on small problems in the three operator modes and checks that
every problem returns its device memory.  A sanitizer report or a failed
expectation gives a non-zero exit status.  build() makes the executable.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "host", "capi_san")
ENV = dict(os.environ, ASAN_OPTIONS="protect_shadow_gap=0:detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run():
    if not os.path.exists(EXE):
        pytest.skip("tests/host/capi_san is not built (run __graft_entry__.build())")
    return subprocess.run([EXE], capture_output=True, text=True, env=ENV, timeout=240)


def test_abi_argument_checks_under_sanitizers():
    env = dict(ENV, HIP_VISIBLE_DEVICES="-1")  # no device: the argument checks alone
    if not os.path.exists(EXE):
        pytest.skip("tests/host/capi_san is not built (run __graft_entry__.build())")
    res = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=240)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "argument checks" in res.stdout and "done" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr


@pytest.mark.gpu
def test_abi_all_entry_points_under_sanitizers():
    print("[gpu-case] sanitized C-ABI driver", flush=True)
    res = _run()
    assert res.returncode == 0, res.stdout + res.stderr
    for mode in (0, 1, 2):
        assert f"operator mode {mode}:" in res.stdout, res.stdout
    assert "projected problem" in res.stdout and res.stdout.strip().endswith("done"), res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
