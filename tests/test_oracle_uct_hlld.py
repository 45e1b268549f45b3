"""Pins of the UCT-HLLD corner EMF (Sec. 2.4 lists the HLLD 2D Riemann solver of
Mignone & Del Zanna 2021 among its edge-EMF schemes).

* The face coefficients: across one face the HLLD flux of a tangential field
  component, written with the oracle's coefficients as
  aL u_L B_L + aR u_R B_R - (dR B_R - dL B_L) - B_n (aL v_L + aR v_R),
  equals the HLLD flux itself (computed by the oracle's HLLD solver, which is
  pinned against textbook properties in test_oracle_pins.py), in every region
  of the fan (each is hit and counted), for B_n = 0 and tiny B_n, with
  aL + aR = 1.
* Plane-parallel reduction along x, y and z: on data that vary along one axis
  only, the edge solve reduces to the 1-D HLLD flux of the tangential field;
  the full 3-D run equals an independent 1-D finite-volume run in numpy (all
  seven fluxes from HLLD) to round-off.
* A fully three-dimensional state relabelled x -> y -> z gives the relabelled
  result; div B stays at round-off and the field totals are conserved.
* Smooth linear waves converge like E^c (errors within 20 %), and the scheme
  differs from UCT-HLL and from E^c in 3-D.
"""
import math

import numpy as np
import pytest

import oracle as O
from helpers import linear_wave_error, linear_wave_modes, permute_xyz, run_to
from paper_2304_13746_amd import inputs as I

GAMMA = 5.0 / 3.0
LINE = ("rho", "mx", "my", "mz", "en", "by", "bz")


def _states(rng, n):
    w = np.zeros((n, 7))
    w[:, 0] = rng.uniform(0.2, 2.0, n)
    w[:, 1] = rng.uniform(-3.0, 3.0, n)
    w[:, 2:4] = rng.normal(0.0, 1.0, (n, 2))
    w[:, 4:6] = rng.normal(0.0, 1.0, (n, 2))
    w[:, 6] = rng.uniform(0.1, 2.0, n)
    return w


def test_coefficients_reproduce_the_hlld_field_flux_in_every_region():
    rng = np.random.default_rng(2021)
    n = 20000
    wl, wr = _states(rng, n), _states(rng, n)
    bn = rng.normal(0.0, 1.0, n)
    bn[:1000] = 0.0
    bn[1000:2000] *= 1e-9
    # degenerate star states: B_t = 0 on both sides with B_n^2 = rho (S - u)^2
    # is not hit by random data; zero tangential field makes den = t - B_n^2
    # vanish where the fast speed equals the Alfven speed
    wl[2000:2500, 4:6] = 0.0
    wr[2000:2500, 4:6] = 0.0
    f, _ = O.riemann(O.HLLD, GAMMA, wl, wr, bn)
    c = O.uct_hlld_coef(GAMMA, wl, wr, bn)
    al, ar, dl, dr = c.T
    assert np.all(al + ar == 1.0)
    for t, (vi, bi) in enumerate(((2, 4), (3, 5))):
        terms = [al * wl[:, 1] * wl[:, bi], ar * wr[:, 1] * wr[:, bi], -dr * wr[:, bi],
                 dl * wl[:, bi], -bn * (al * wl[:, vi]), -bn * (ar * wr[:, vi])]
        pred = (terms[0] + terms[1]) + (terms[2] + terms[3]) + (terms[4] + terms[5])
        scale = sum(np.abs(x) for x in terms) + np.abs(f[:, 5 + t]) + 1e-300
        err = np.abs(pred - f[:, 5 + t]) / scale
        assert float(np.max(err)) <= 1e-13, (t, float(np.max(err)))
    # every region of the fan occurs: L and R (aL or aR = 1, no diffusion), the
    # single-star regions (one-sided diffusion), the double-star ones (0 < aR < 1)
    one_l, one_r = (al == 1.0) & (ar == 0.0), (al == 0.0) & (ar == 1.0)
    regions = {"L": one_l & (dl == 0) & (dr == 0), "*L": one_l & (dl != 0),
               "**": ~one_l & ~one_r, "*R": one_r & (dr != 0), "R": one_r & (dl == 0) & (dr == 0)}
    counts = {k: int(np.count_nonzero(v)) for k, v in regions.items()}
    print(counts)
    assert all(v > 100 for v in counts.values()), counts
    # B_n = 0: no double-star region (S*_L = S_M = S*_R)
    assert not np.any(regions["**"][:1000])
    # the double-star weights stay bounded for tiny B_n
    assert np.all((al >= -1e-12) & (al <= 1 + 1e-12))


def _vl(dm, dp):
    out = np.zeros_like(dm)
    m = dm * dp > 0
    out[m] = 2.0 * dm[m] * dp[m] / (dm[m] + dp[m])
    return out


def _rhs_1d(u, bx, dx):
    """-dF/dx on a periodic line with PLM and every flux from HLLD;
    u = (rho, mx, my, mz, E, By, Bz), shape (7, n)."""
    rho, mx, my, mz, en, by, bz = u
    vx, vy, vz = mx / rho, my / rho, mz / rho
    p = (GAMMA - 1.0) * (en - 0.5 * (mx * vx + my * vy + mz * vz) - 0.5 * (bx * bx + by * by + bz * bz))
    w = np.stack([rho, vx, vy, vz, by, bz, p])
    sl = _vl(w - np.roll(w, 1, axis=1), np.roll(w, -1, axis=1) - w)
    wl = w + 0.5 * sl
    wr = np.roll(w - 0.5 * sl, -1, axis=1)
    f, _ = O.riemann(O.HLLD, GAMMA, wl.T, wr.T, np.full(rho.size, bx))
    f = f.T
    return -(f - np.roll(f, 1, axis=1)) / dx


def _tube(n, m):
    x = (np.arange(n) + 0.5) / n
    left = np.abs(x - 0.5) < 0.25
    rho = np.where(left, 1.0, 0.125)
    pr = np.where(left, 1.0, 0.1)
    by = np.where(left, 1.0, -1.0)
    bz = np.where(left, 0.2, 0.5)
    vy = np.where(left, 0.1, -0.3)
    vz = np.where(left, -0.2, 0.15)
    return I.assemble(rho, 0.05, vy, vz, pr, 0.75, by, bz, GAMMA, shape=(m, m, n)), 0.75


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_parallel_reduction_every_axis(axis):
    n, m, cycles = 64, 2, 6
    s, bx = _tube(n, m)
    dx = 1.0 / n
    dt = 0.2 * dx
    ref = np.stack([s[f][0, 0] for f in LINE])
    for _ in range(cycles):
        u1 = ref + dt * _rhs_1d(ref, bx, dx)
        ref = 0.5 * (u1 + dt * _rhs_1d(u1, bx, dx)) + 0.5 * ref
    g = s
    dims, ls = [n, m, m], [1.0, m * dx, m * dx]
    for _ in range(axis):
        g = permute_xyz(g)
        dims = [dims[2], dims[0], dims[1]]
        ls = [ls[2], ls[0], ls[1]]
    g = O.copy_state(g)
    p = O.Params(*dims, *ls, riemann=O.HLLD, emf=O.EMF_UCT_HLLD)
    for _ in range(cycles):
        O.step(p, g, 0.0, dt, 1)
    for _ in range((3 - axis) % 3):
        g = permute_xyz(g)
    got = np.stack([g[f][0, 0] for f in LINE])
    scale = np.max(np.abs(ref), axis=1, keepdims=True)
    err = float(np.max(np.abs(got - ref) / scale))
    print("axis", axis, "max rel", err)
    assert err <= 1e-12
    # the field components vary along the line only: nothing leaks sideways
    for f in LINE:
        assert np.max(np.abs(g[f] - g[f][0:1, 0:1, :])) <= 1e-14 * max(1.0, np.max(np.abs(g[f])))


def test_cyclic_axis_permutation_3d():
    n = 16
    s = I.orszag_tang_3d(n)
    dt = 0.1 / n
    outs = []
    for st in (s, permute_xyz(s)):
        st = O.copy_state(st)
        p = O.Params(n, n, n, riemann=O.HLLD, emf=O.EMF_UCT_HLLD)
        for _ in range(6):
            O.step(p, st, 0.0, dt, 1)
        outs.append(st)
    a = permute_xyz(outs[0])
    for f in O.FIELDS:
        assert np.max(np.abs(a[f] - outs[1][f])) <= 1e-12 * max(1.0, np.max(np.abs(a[f]))), f


def test_divb_totals_and_difference_from_other_schemes():
    dims = (20, 12, 16)
    s = I.turbulence(dims, seed=5, kpeak=2.0, mach=1.0, b0=(0.2, -0.3, 0.1))
    l = s.pop("_l")
    p = O.Params(*dims, *l, emf=O.EMF_UCT_HLLD, integrator=O.RK3)
    d0 = O.diagnostics(p, s)
    out = {}
    for emf in (O.EMF_UCT_HLLD, O.EMF_UCT_HLL, O.EMF_EC):
        st = O.copy_state(s)
        O.step(O.Params(*dims, *l, emf=emf, integrator=O.RK3), st, 0.0, 0.0, 10)
        out[emf] = st
    st = out[O.EMF_UCT_HLLD]
    d = O.diagnostics(p, st)
    bmax = max(float(np.max(np.abs(st[f]))) for f in ("bx", "by", "bz"))
    assert d["divb_max"] / max(dims) / bmax <= 1e-14
    assert np.allclose(d["bflux"], d0["bflux"], rtol=0, atol=1e-13)
    assert abs(d["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    assert abs(d["energy"] - d0["energy"]) <= 1e-13 * abs(d0["energy"])
    for other in (O.EMF_UCT_HLL, O.EMF_EC):
        assert np.max(np.abs(out[other]["bx"] - st["bx"])) > 1e-6 * bmax


@pytest.mark.parametrize("wave", ["fast", "alfven"])
def test_linear_waves_converge_like_ec(wave):
    """Sec. 4.2 linear waves on the inclined 2N x N x N box, one crossing time:
    the error falls by a factor >= 2^(2 x 1.6) from N = 8 to 32 and at N = 32 it
    is within 20 % of the E^c error."""
    errs = []
    for n in (8, 16, 32):
        s, info = I.linear_wave(wave, n)
        s0 = O.copy_state(s)
        p = O.Params(*info["dims"], *info["l"], gamma=GAMMA, cfl=0.3, emf=O.EMF_UCT_HLLD)
        run_to(p, s, 1.0 / abs(info["speed"]))
        errs.append(linear_wave_error(s0, s, info["eps"], linear_wave_modes(info)))
    p = O.Params(*info["dims"], *info["l"], gamma=GAMMA, cfl=0.3, emf=O.EMF_EC)
    st, _ = I.linear_wave(wave, 32)
    run_to(p, st, 1.0 / abs(info["speed"]))
    e_ec = linear_wave_error(s0, st, info["eps"], linear_wave_modes(info))
    slope = math.log2(errs[0] / errs[2]) / 2
    print(wave, errs, slope, e_ec)
    assert slope >= 1.6, (errs, slope)
    assert abs(errs[2] - e_ec) <= 0.2 * e_ec, (errs[2], e_ec)


def test_parameter_checks():
    s = I.orszag_tang(8)
    for kw in ({"riemann": O.HLLC}, {"riemann": O.HLL}):
        p = O.Params(8, 8, 8, emf=O.EMF_UCT_HLLD, **kw)
        with pytest.raises(RuntimeError):
            O.step(p, O.copy_state(s), 0.0, 0.0, 1)


def test_rotation_by_pi_about_z():
    """(x, y) -> (-x, -y) commutes with the scheme to round-off: an edge flux
    combines the coefficients of the two faces it crosses symmetrically (a
    combination that favours one of them breaks this)."""
    from helpers import rotate_pi_z
    dims = (16, 16, 8)
    s = I.turbulence(dims, seed=9, kpeak=2.0, mach=1.0, b0=(0.2, -0.3, 0.1))
    l = s.pop("_l")
    p = O.Params(*dims, *l, emf=O.EMF_UCT_HLLD)
    a, b = O.copy_state(s), O.copy_state(rotate_pi_z(s))
    O.step(p, a, 0.0, 0.0, 4)
    O.step(p, b, 0.0, 0.0, 4)
    ra = rotate_pi_z(a)
    for f in O.FIELDS:
        assert np.max(np.abs(ra[f] - b[f])) <= 1e-12 * max(1.0, np.max(np.abs(b[f]))), f
