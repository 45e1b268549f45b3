"""The cell-index helpers of the UCT and vector-potential kernels, compiled for
the host: cell coordinates from a linear index and periodic stencil wraps equal
the plain modulo formulas on narrow, ragged, cubic and more-than-2^31-cell boxes
(the last ones take the 64-bit branch, which no GPU test can allocate)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cstdio>
#include <random>
#include "mhd_internal.h"
int main() {
  std::mt19937_64 g(7);
  long bad = 0, checked = 0;
  const long long dims[][3] = {{1, 1, 33}, {2, 9, 5}, {33, 1, 1}, {37, 29, 11}, {1, 1, 1},
                               {256, 256, 256}, {4096, 2, 3}, {3, 4096, 2}, {512, 512, 512},
                               {2048, 2048, 600}, {4096, 4096, 200}};
  for (const auto& d : dims) {
    const long long nx = d[0], ny = d[1], nz = d[2], plane = nx * ny, n = plane * nz;
    for (int t = 0; t < 100000; ++t) {
      // the first and last cells, then seeded samples
      const long long c = t < 50 ? t % n : (t < 100 ? n - 1 - (t - 50) % n : (long long)(g() % n));
      int i, j, k;
      mhd::cell_ijk(c, (int)nx, plane, n, i, j, k);
      if (i != c % nx || j != (c / nx) % ny || k != c / plane) ++bad;
      for (int o = -3; o <= 3; ++o) {
        if (mhd::wrap_index(i + o, (int)nx) != (int)(((i + o) % nx + nx) % nx)) ++bad;
        if (mhd::wrap_index(j + o, (int)ny) != (int)(((j + o) % ny + ny) % ny)) ++bad;
        if (mhd::wrap_index(k + o, (int)nz) != (int)(((k + o) % nz + nz) % nz)) ++bad;
      }
      ++checked;
    }
  }
  printf("%ld %ld\n", checked, bad);
  return 0;
}
"""


def test_index_helpers_match_modulo(tmp_path):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = tmp_path / "idx.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "idx"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-w",
                           "-I" + os.path.join(ROOT, "paper_2304_13746_amd", "csrc"),
                           str(src), "-o", str(exe)])
    checked, bad = map(int, subprocess.check_output([str(exe)]).decode().split())
    assert checked == 11 * 100000
    assert bad == 0
