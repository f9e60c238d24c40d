"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/host_sanitizer_driver.cpp exercises the host logic: argument validation of the constructors,
error reporting, the Daubechies filters, the FFT twiddle and Bluestein tables (checked against
their definitions in FP64), and context creation without a device.  The sanitized library is
rebuilt when a source changed since the last build.  The test runs where no GPU is visible: the
device runtime is then reduced to its error paths, which are part of what is checked.
"""
import glob
import hashlib
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STAMP_DIR = os.path.join(ROOT, "paper_1602_08847_amd", "_build", "hostsan")


def sources_digest() -> str:
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1602_08847_amd", "csrc", "*")))
    files += [os.path.join(ROOT, "include", "muffin.h"), os.path.join(ROOT, "tests", "host_sanitizer_driver.cpp"),
              os.path.join(ROOT, "paper_1602_08847_amd", "build.py")]
    h = hashlib.sha256()
    for f in files:
        h.update(f.encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def test_host_code_is_clean_under_asan_and_ubsan():
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("host sanitizer checks run where no GPU is visible")
    from paper_1602_08847_amd import build
    digest = sources_digest()
    stamp = os.path.join(STAMP_DIR, "digest")
    exe = os.path.join(STAMP_DIR, "host_sanitizer_driver")
    if not (os.path.exists(exe) and os.path.exists(stamp) and open(stamp).read() == digest):
        exe = build.build_host_sanitized()
        with open(stamp, "w") as f:
            f.write(digest)
    env = dict(os.environ)
    # the device runtime keeps allocations for the process's lifetime: leak reports are not findings
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "host checks passed" in r.stdout
