"""The C ABI under host AddressSanitizer and UndefinedBehaviorSanitizer.

`python -m paper_2404_07293_amd.build --sanitize` (also run by
__graft_entry__.build) compiles every library source with the host pass
instrumented and links the driver tests/sanitize/abi_check.cpp. The driver
walks the ABI's validation paths (here, without a device) and, on a GPU,
full solves on both boundary routes, a batch with the device eigensolver,
syntheses in every form, a batched sweep and the surrogate. A sanitizer report
aborts the driver (undefined behaviour is not recovered from); the banners
are checked as well."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2404_07293_amd", "_build_san", "abi_check")
BANNERS = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:")


def run(mode, leaks):
    if not os.path.exists(EXE):
        pytest.skip("sanitizer driver not built (python -m paper_2404_07293_amd.build --sanitize)")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=%d:abort_on_error=1" % (1 if leaks else 0)
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([EXE, mode], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert r.returncode == 0, out[-4000:]
    for b in BANNERS:
        assert b not in out
    assert "0 failure(s)" in r.stdout


def test_abi_validation_paths_under_sanitizers():
    """No device: every entry point rejects null or out-of-range arguments
    and reports the error; no memory error, no undefined behaviour, no
    leak."""
    run("cpu", leaks=True)


@pytest.mark.gpu
def test_abi_device_paths_under_sanitizers():
    """On a GPU: solves, syntheses, batch, surrogate and error paths with the
    host code instrumented. Leak detection is off here: the HIP runtime keeps
    allocations of its own until the process ends."""
    run("gpu", leaks=False)
