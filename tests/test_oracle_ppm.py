"""Pins of the PPM reconstruction (Sec. 2.3: Colella & Woodward 1984 with the
extremum-preserving limiter of Colella & Sekora 2008).

* The interface value 7/12 (a_j + a_{j+1}) - 1/12 (a_{j-1} + a_{j+2}) is exact
  for cubics: on cell averages of a smooth monotone cubic the face values are
  the cubic's point values.
* At a smooth extremum the limiter keeps that accuracy (the property the
  limiter exists for): cell averages of a parabola around its vertex give its
  exact face values, where a classic PPM flattening would not.
* A step gains no overshoot; monotone data stay bounded.
* On the linear waves of Sec. 4.2, PPM + RK3 has a lower error than van Leer +
  RK2 at the resolutions where the paper shows it ahead.
"""
import numpy as np
import pytest

import oracle as O
from helpers import linear_wave_error, linear_wave_modes
from paper_2304_13746_amd import inputs as I


def cell_avg(coef, xc, h):
    """Exact cell average of sum_k coef[k] x^k over [xc - h/2, xc + h/2]."""
    lo, hi = xc - h / 2, xc + h / 2
    return sum(c * (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k, c in enumerate(coef)) / h


def poly(coef, x):
    return sum(c * x ** k for k, c in enumerate(coef))


def test_exact_for_monotone_cubics():
    rng = np.random.default_rng(12)
    h = 0.05
    done = 0
    for _ in range(400):
        coef = [rng.normal(), 1.0 + rng.uniform(0, 1), 0.3 * rng.normal(), 0.3 * rng.normal()]
        x0 = rng.uniform(-0.5, 0.5)
        a = [cell_avg(coef, x0 + (k - 2) * h, h) for k in range(5)]
        if np.any(np.diff(a) <= 0):
            continue  # keep to strictly monotone data
        lo, hi = O.ppm_faces(a)
        assert abs(hi - poly(coef, x0 + h / 2)) <= 1e-12
        assert abs(lo - poly(coef, x0 - h / 2)) <= 1e-12
        done += 1
    assert done > 100


def test_smooth_extremum_is_not_clipped():
    h = 0.05
    for x0 in (0.0, 0.01, -0.02):
        coef = [0.3, 0.0, 1.0]  # vertex at x = 0
        a = [cell_avg(coef, x0 + (k - 2) * h, h) for k in range(5)]
        lo, hi = O.ppm_faces(a)
        assert abs(hi - poly(coef, x0 + h / 2)) <= 1e-12
        assert abs(lo - poly(coef, x0 - h / 2)) <= 1e-12


def test_step_and_monotone_bounds():
    assert O.ppm_faces([0.0, 0.0, 0.0, 1.0, 1.0]) == (0.0, 0.0)
    assert O.ppm_faces([0.0, 0.0, 1.0, 1.0, 1.0]) == (1.0, 1.0)
    rng = np.random.default_rng(5)
    for _ in range(500):
        a = np.sort(rng.normal(size=5)) * rng.choice([-1, 1])
        lo, hi = O.ppm_faces(a)
        b0, b1 = min(a[1], a[3]), max(a[1], a[3])
        assert b0 - 1e-14 <= lo <= b1 + 1e-14 and b0 - 1e-14 <= hi <= b1 + 1e-14


@pytest.mark.parametrize("wave", ["fast", "alfven"])
def test_ppm_rk3_linear_waves(wave):
    def err(n, recon, integ):
        s0, info = I.linear_wave(wave, n)
        s = O.copy_state(s0)
        p = O.Params(*info["dims"], *info["l"], integrator=integ, recon=recon)
        t_end = 1.0 / abs(info["speed"])  # one wavelength (|k| = 2 pi)
        t, dt = 0.0, 0.0
        while t < t_end:
            t, dt, _ = O.step(p, s, t, dt, 1, t_end)
        return linear_wave_error(s0, s, info["eps"], linear_wave_modes(info))

    e_plm = [err(n, O.PLM, O.RK2) for n in (8, 16)]
    e_ppm = [err(n, O.PPM, O.RK3) for n in (8, 16)]
    print(wave, "plm+rk2", e_plm, "ppm+rk3", e_ppm)
    assert e_ppm[0] < e_plm[0] and e_ppm[1] < e_plm[1]
