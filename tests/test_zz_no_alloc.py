"""The allocation-free diagnostics entry point (mhd_get_diagnostics_noalloc):
through the C ABI, two calls in a row on two boxes, the second smaller, each
bit-identical to mhd_get_diagnostics on the same state (same kernels, same
summation order; only the partial-sum rows live elsewhere)."""
import ctypes as C

import pytest

from gpu_util import gpu_box, need_gpu
from paper_2304_13746_amd import _lib as L
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu


def _diag(box, name):
    d = L.Diag()
    L.check(getattr(box.lib, name)(box.ctx, C.byref(d)), name)
    return (d.mass, tuple(d.mom), d.energy, tuple(d.bflux), d.divb_max, d.divb_rms, d.status)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_diagnostics_equal_workspace_diagnostics(precision):
    need_gpu()
    results = []
    for n in (40, 24):  # the second call on a smaller box
        print(f"noalloc diagnostics {precision} {n}^3", flush=True)
        s = I.orszag_tang(n)
        if precision == "fp32":
            s = I.to_float32_exact(s)
        box = gpu_box((n, n, n), precision=precision)
        box.set_state(s)
        box.step(2)
        a = _diag(box, "mhd_get_diagnostics_noalloc")
        b = _diag(box, "mhd_get_diagnostics")
        assert a == b, (n, a, b)
        assert a[-1] == 0 and a[0] > 0
        results.append(a)
        box.close()
    assert results[0] != results[1]
    # a null argument is an argument error, not a fault
    lib = L.lib()
    assert lib.mhd_get_diagnostics_noalloc(None, None) == L.MHD_ERR_INVALID_ARG
