"""The oracle and the operation counter under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only): the oracle's C source built with
-fsanitize=address,undefined (undefined behaviour aborts) runs a broad set of
the oracle pins in a child process, and the counter built the same way runs on
a seeded input with leak detection on.  Any out-of-bounds access, use after
free, leak (counter) or undefined operation fails the test."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from paper_2304_13746_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
# pin files that exercise every oracle path in about a minute under the sanitizers
PINS = ["test_oracle_pins.py", "test_oracle_diag.py", "test_oracle_emf.py", "test_oracle_limo3.py",
        "test_oracle_ppm.py", "test_oracle_vpot.py", "test_oracle_sedov.py", "test_fp32_ties.py",
        "test_serve_sched.py"]


def _libasan():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++") or not _libasan():
        pytest.skip("gcc with the address sanitizer runtime is not available")
    d = tmp_path_factory.mktemp("san")
    lib = str(d / "liborc_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                           "-fPIC", "-shared", "-std=c11", *SAN, "-o", lib,
                           os.path.join(ROOT, "oracle", "mhd_oracle.c"), "-lm"])
    exe = str(d / "opcount_san")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fpermissive", "-w", *SAN,
                           "-I" + os.path.join(ROOT, "oracle"), "-o", exe,
                           os.path.join(ROOT, "oracle", "opcount.cpp")])
    return d, lib, exe


def test_oracle_pins_under_sanitizers(sanitized):
    d, lib, _ = sanitized
    env = dict(os.environ, MHD_ORACLE_LIB=lib, LD_PRELOAD=_libasan(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", f) for f in PINS]],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_operation_counter_under_sanitizers(sanitized):
    d, _, exe = sanitized
    s = I.turbulence(12, seed=2304, kpeak=3.0, mach=0.5, b0=(0.2, 0.0, 0.0))
    s.pop("_l")
    f = d / "st.bin"
    np.concatenate([s[k].ravel() for k in ("rho", "mx", "my", "mz", "en", "bx", "by", "bz")]
                   ).astype(np.float64).tofile(f)
    for extra in ((), ("hll",)):
        r = subprocess.run([exe, str(f), "12", "12", "12", *extra], capture_output=True, text=True,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"), timeout=300)
        assert r.returncode == 0, r.stderr[-3000:]
        assert '"method_flops"' in r.stdout
