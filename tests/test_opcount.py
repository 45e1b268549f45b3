"""The algorithmic operation counter (oracle/opcount.cpp) that the benchmark's
ALU roofline uses: it builds, and its counts follow the method's structure."""
import json
import os
import subprocess

import numpy as np
import pytest

from paper_2304_13746_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def opcount(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("opc") / "opcount")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fpermissive", "-w",
                           "-I" + os.path.join(ROOT, "oracle"), "-o", exe,
                           os.path.join(ROOT, "oracle", "opcount.cpp")])
    return exe


def count(exe, tmp_path, s, n, solver=()):
    raw = np.concatenate([s[k].ravel() for k in ("rho", "mx", "my", "mz", "en", "bx", "by", "bz")])
    f = tmp_path / "st.bin"
    raw.astype(np.float64).tofile(f)
    out = subprocess.check_output([exe, str(f), str(n), str(n), str(n), *solver]).decode()
    return json.loads(out)


def test_counts_follow_the_method(opcount, tmp_path):
    s = I.turbulence(16, seed=2304, kpeak=4.0, mach=0.5, b0=(0.2, 0.0, 0.0))
    s.pop("_l")
    d = count(opcount, tmp_path, s, 16)
    h = count(opcount, tmp_path, s, 16, ("hll",))
    # square roots: per face two fast speeds (2 each) + HLLD's two star densities
    assert d["sqrt"] == 18.0 and h["sqrt"] == 12.0
    # divisions: 1/rho per cell, 14 + 7 + 7... at least the 21 limiter slopes
    # evaluated by the oracle on 3 faces x 14 (minus those cut by sign tests)
    assert d["div"] > 20 and h["div"] < d["div"]
    assert 1100 < d["flops"] < 1500 and h["flops"] < d["flops"]


def test_uniform_state_counts_no_limiter_divisions(opcount, tmp_path):
    """On a uniform state every one-sided difference is zero, so no van Leer
    division is taken: the divisions left are 1/rho (S1) plus the Riemann ones."""
    s = I.assemble(1.0, 0.1, 0.2, 0.3, 0.6, 0.2, 0.1, 0.05, 5.0 / 3.0, shape=(8, 8, 8))
    h = count(opcount, tmp_path, s, 8, ("hll",))
    # HLL: per face 2 x (1/rho in the fast speed) + 1/(S_R - S_L) = 3; 3 faces; S1: 1
    assert h["div"] == 10.0


def test_repeated_slope_work_is_the_lower_face_reconstruction(opcount, tmp_path):
    """The count without repeated work drops, per cell, direction and
    reconstructed variable, the lower-face pass over differences and slope the
    upper face already formed: on a uniform state (zero differences, van Leer
    returns 0 after its one product) that pass is 2 differences + 1 product +
    1 halving + 1 subtraction = 5 operations, for 7 variables and 3 directions."""
    s = I.assemble(1.0, 0.1, 0.2, 0.3, 0.6, 0.2, 0.1, 0.05, 5.0 / 3.0, shape=(8, 8, 8))
    h = count(opcount, tmp_path, s, 8, ("hll",))
    assert h["repeated"] == 5 * 7 * 3
    assert h["method_flops"] == pytest.approx(h["flops"] - h["repeated"], abs=0.01)
    t = I.turbulence(16, seed=2304, kpeak=4.0, mach=0.5, b0=(0.2, 0.0, 0.0))
    t.pop("_l")
    d = count(opcount, tmp_path, t, 16)
    # with non-zero slopes the repeated pass also holds van Leer's remaining
    # product, sum and division: between 5 and 8 operations per variable
    assert 5 * 21 < d["repeated"] <= 8 * 21
