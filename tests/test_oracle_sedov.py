"""Pins of the hydrodynamic workload: the Sedov-Taylor blast of Sec. 4.1
(rho = 1, P = 1e-2, gamma = 5/3, E = 1 deposited in a small sphere, periodic
unit cube, HLL or HLLC, RK2, PLM, B = 0).

* The shock follows the self-similar Sedov-Taylor radius
  R(t) = xi_0 (E t^2 / rho)^(1/5), xi_0 = 1.152 for gamma = 5/3 in three
  dimensions (Sedov 1959), to a few per cent already on a 32^3 grid.
* Mass and total energy are conserved to round-off; the field stays zero.
"""
import numpy as np
import pytest

import oracle as O
from paper_2304_13746_amd import inputs as I

XI0 = 1.152


def shock_radius(rho, n):
    """Radius of the peak of the angle-averaged density."""
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h - 0.5
    r = np.sqrt(x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2)
    rb = np.round(r / h).astype(int).ravel()
    cnt = np.bincount(rb)
    prof = np.where(cnt > 0, np.bincount(rb, weights=rho.ravel()) / np.maximum(cnt, 1), 0.0)
    return float(np.argmax(prof)) * h


@pytest.mark.parametrize("solver", [O.HLL, O.HLLC])
def test_sedov_radius_and_conservation(solver):
    n = 32
    s = I.sedov(n)
    p = O.Params(n, n, n, riemann=solver)
    d0 = O.diagnostics(p, s)
    radii = []
    t, dt = 0.0, 0.0
    for t_end in (0.02, 0.05):
        while t < t_end:
            t, dt, _ = O.step(p, s, t, dt, 1, t_end)
        assert t == pytest.approx(t_end, rel=1e-14)
        radii.append(shock_radius(s["rho"], n))
        r_th = XI0 * (1.0 * t_end ** 2) ** 0.2
        assert abs(radii[-1] / r_th - 1.0) < 0.06, (t_end, radii[-1], r_th)
    d1 = O.diagnostics(p, s)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    assert abs(d1["energy"] - d0["energy"]) <= 1e-13 * d0["energy"]
    assert np.all(np.abs(d1["mom"]) <= 1e-13)
    for f in ("bx", "by", "bz"):
        assert not s[f].any()
