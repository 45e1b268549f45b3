"""Pins of the corner-EMF schemes of Sec. 2.4 (E^c, E^0, arithmetic average of
Gardiner & Stone 2005).

* Any scheme keeps div B at round-off (constrained transport does not depend
  on how the edge EMF is built).
* On plane-parallel data (variation along x only) E^c and E^0 reduce the
  3-D constrained-transport scheme to the 1-D Godunov scheme: the result
  equals an independent 1-D finite-volume run (cell-centred B_t, same PLM,
  same face Riemann solver, same RK2 cycle) written below with numpy.  The
  arithmetic average does not reduce (its known defect), so it differs there.
"""
import numpy as np
import pytest

import oracle as O
from paper_2304_13746_amd import inputs as I

GAMMA = 5.0 / 3.0


@pytest.mark.parametrize("emf", [O.EMF_EC, O.EMF_E0, O.EMF_ARITH])
def test_divb_stays_at_roundoff(emf):
    n = 16
    s = I.orszag_tang_3d(n)
    p = O.Params(n, n, n, emf=emf)
    O.step(p, s, 0.0, 0.0, 8)
    d = O.diagnostics(p, s)
    bmax = max(float(np.max(np.abs(s[f]))) for f in ("bx", "by", "bz"))
    assert d["divb_max"] / n / bmax <= 1e-14


def _vl(dm, dp):
    # harmonic van Leer slope, written independently of the oracle
    out = np.zeros_like(dm)
    m = dm * dp > 0
    out[m] = 2.0 * dm[m] * dp[m] / (dm[m] + dp[m])
    return out


def _rhs_1d(u, bx, dx, riemann):
    """-dF/dx of the 1-D ideal-MHD system on a periodic line of cells;
    u = (rho, mx, my, mz, E, By, Bz) cell averages, shape (7, n)."""
    rho, mx, my, mz, en, by, bz = u
    vx, vy, vz = mx / rho, my / rho, mz / rho
    p = (GAMMA - 1.0) * (en - 0.5 * (mx * vx + my * vy + mz * vz) - 0.5 * (bx * bx + by * by + bz * bz))
    w = np.stack([rho, vx, vy, vz, by, bz, p])
    dm = w - np.roll(w, 1, axis=1)
    dp = np.roll(w, -1, axis=1) - w
    sl = _vl(dm, dp)
    wl = (w + 0.5 * sl)                       # left state of face i+1/2
    wr = np.roll(w - 0.5 * sl, -1, axis=1)    # right state of face i+1/2
    n = rho.size
    f, _ = O.riemann(riemann, GAMMA, wl.T, wr.T, np.full(n, bx))
    f = f.T  # (rho, m_n, m_t1, m_t2, E, B_t1, B_t2) at faces i+1/2
    return -(f - np.roll(f, 1, axis=1)) / dx


def _rk2_1d(u, bx, dx, dt, cycles, riemann):
    for _ in range(cycles):
        u1 = u + dt * _rhs_1d(u, bx, dx, riemann)
        u = 0.5 * (u1 + dt * _rhs_1d(u1, bx, dx, riemann)) + 0.5 * u
    return u


@pytest.mark.parametrize("riemann", [O.HLLD, O.HLL])
def test_plane_parallel_reduction(riemann):
    n, m = 64, 2
    x = (np.arange(n) + 0.5) / n
    left = np.abs(x - 0.5) < 0.25
    rho = np.where(left, 1.0, 0.125)
    pr = np.where(left, 1.0, 0.1)
    by = np.where(left, 1.0, -1.0)
    bz = np.where(left, 0.2, 0.5)
    vy = np.where(left, 0.1, -0.3)
    bx = 0.75
    sh = (m, m, n)
    s = I.assemble(rho, 0.05, vy, 0.0, pr, bx, by, bz, GAMMA, shape=sh)
    dx = 1.0 / n
    dt = 0.2 * dx
    # the same line as 1-D cell averages (y- and z-uniform face fields equal the cell values)
    u = np.stack([s["rho"][0, 0], s["mx"][0, 0], s["my"][0, 0], s["mz"][0, 0], s["en"][0, 0],
                  s["by"][0, 0], s["bz"][0, 0]])
    ref = _rk2_1d(u, bx, dx, dt, 6, riemann)
    errs = {}
    for emf in (O.EMF_EC, O.EMF_E0, O.EMF_ARITH):
        g = O.copy_state(s)
        p = O.Params(n, m, m, 1.0, m * dx, m * dx, riemann=riemann, emf=emf)
        for _ in range(6):
            O.step(p, g, 0.0, dt, 1)
        got = np.stack([g[f][0, 0] for f in ("rho", "mx", "my", "mz", "en", "by", "bz")])
        scale = np.max(np.abs(ref), axis=1, keepdims=True)
        errs[emf] = float(np.max(np.abs(got - ref) / scale))
    print(errs)
    assert errs[O.EMF_EC] <= 1e-12, errs
    assert errs[O.EMF_E0] <= 1e-12, errs
    assert errs[O.EMF_ARITH] > 1e-4, errs


def test_scheme_building_blocks():
    """E^0 is E^c with every switch at its tie; the arithmetic scheme ignores
    the cell EMFs and mass fluxes; all three agree on uniform data."""
    rng = np.random.default_rng(4)
    for _ in range(50):
        a = rng.normal(size=8)
        sgn = rng.normal(size=4)
        e0 = O.corner_emf_scheme(O.EMF_E0, *a, *sgn)
        assert e0 == O.corner_emf(*a, 0.0, 0.0, 0.0, 0.0)
        ar = O.corner_emf_scheme(O.EMF_ARITH, *a, *sgn)
        assert ar == O.corner_emf_scheme(O.EMF_ARITH, *a[:4], 0, 0, 0, 0, 1, 1, 1, 1)
        assert O.corner_emf_scheme(O.EMF_EC, *a, *sgn) == O.corner_emf(*a, *sgn)
    u = [0.7] * 8
    vals = {O.corner_emf_scheme(k, *u, 1.0, -1.0, 0.5, -0.5) for k in (0, 1, 2)}
    assert vals == {0.7}
