"""A plain host program (paper_2304_13746_amd/csrc/mhd_abi_example.cpp) that
uses only include/mhd.h and the HIP runtime advances a box through the C ABI;
its result is bit-identical to the oracle (FP64)."""
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from gpu_util import FIELDS, need_gpu
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2304_13746_amd", "mhd_abi_example")


def test_c_caller_matches_oracle(tmp_path):
    need_gpu()
    assert os.path.exists(EXE), "the C ABI example is built with the library"
    dims = (40, 24, 20)
    s = I.turbulence(dims, seed=23, kpeak=2.0, mach=0.9, b0=(0.2, 0.1, -0.2),
                     l=(1.0, 1.0, 1.0))
    s.pop("_l")
    raw = np.concatenate([s[f].ravel() for f in FIELDS])
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    raw.tofile(fin)
    r = subprocess.run([EXE, str(fin), str(fout), *map(str, dims), "4"], capture_output=True,
                       text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    out = np.fromfile(fout, dtype=np.float64)
    n = int(np.prod(dims))
    g = {f: out[q * n:(q + 1) * n].reshape(s["rho"].shape) for q, f in enumerate(FIELDS)}
    t_gpu, dt_gpu = out[8 * n], out[8 * n + 1]
    o = O.copy_state(s)
    t, dt, _ = O.step(O.Params(*dims), o, 0.0, 0.0, 4)
    for f in FIELDS:
        assert np.array_equal(g[f], o[f]), f
    assert t_gpu == t and dt_gpu == dt
