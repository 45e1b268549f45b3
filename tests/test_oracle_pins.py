"""Pins of the oracle's building blocks against facts the paper and the
mathematics fix (no GPU).  Each test names what pins it."""
import math

import numpy as np
import pytest

import oracle as O
from helpers import golden

RNG = np.random.default_rng(12345)


def random_states(n, rng, bfield=True):
    """n random face-frame primitive states (rho, vn, vt1, vt2, Bt1, Bt2, p) and Bn."""
    w = np.empty((n, 7))
    w[:, 0] = rng.uniform(0.1, 3.0, n)
    w[:, 1:4] = rng.uniform(-2.0, 2.0, (n, 3))
    w[:, 4:6] = rng.uniform(-1.5, 1.5, (n, 2)) if bfield else 0.0
    w[:, 6] = rng.uniform(0.05, 3.0, n)
    bn = rng.uniform(-1.5, 1.5, n) if bfield else np.zeros(n)
    return w, bn


def test_wave_speeds_printed_in_paper():
    """Sec. 4.2: at rho = 1, P = 3/5, gamma = 5/3, B1 = 1, B2 = 3/2 the fast,
    Alfven and slow speeds along x1 are 2, 1 and 0.5."""
    g = golden()["linear_wave_background"]
    cf = O.fast_speed(g["gamma"], g["rho"], g["p"], g["B1"], g["B2"], 0.0)
    cs = O.slow_speed(g["gamma"], g["rho"], g["p"], g["B1"], g["B2"], 0.0)
    assert cf == g["c_fast"]
    assert cs == g["c_slow"]
    assert g["B1"] / math.sqrt(g["rho"]) == g["c_alfven"]
    # the speeds bracket: slow <= Alfven (normal) <= fast, fast >= sound speed
    assert cs <= g["c_alfven"] <= cf


def test_fast_speed_limits():
    """B = 0 gives the sound speed; perpendicular field gives sqrt(a^2 + b^2)."""
    for rho, p in [(1.0, 0.6), (0.3, 2.0), (2.5, 0.01)]:
        g = 5.0 / 3.0
        a = math.sqrt(g * p / rho)
        assert O.fast_speed(g, rho, p, 0.0, 0.0, 0.0) == pytest.approx(a, rel=1e-15)
        b = 0.7
        assert O.fast_speed(g, rho, p, 0.0, b, 0.0) == pytest.approx(math.sqrt(a * a + b * b / rho),
                                                                      rel=1e-14)


def test_vanleer_limiter_properties():
    """Sec. 2.3 (van Leer limiter): symmetric, zero at extrema, bounded by twice
    the smaller one-sided difference (TVD), exact for linear data."""
    dm = RNG.normal(size=2000)
    dp = RNG.normal(size=2000)
    for a, b in zip(dm, dp):
        s = O.vanleer(a, b)
        assert s == O.vanleer(b, a)
        if a * b <= 0:
            assert s == 0.0
        else:
            assert np.sign(s) == np.sign(a)
            assert abs(s) <= 2 * min(abs(a), abs(b)) * (1 + 1e-15)
            assert min(abs(a), abs(b)) * (1 - 1e-15) <= abs(s) <= max(abs(a), abs(b)) * (1 + 1e-15)
    for a in [0.5, -3.0, 1e-7]:
        assert O.vanleer(a, a) == pytest.approx(a, rel=2e-16)


@pytest.mark.parametrize("solver", [O.HLLD, O.HLL])
def test_riemann_consistency(solver):
    """A Riemann solver fed identical left and right states returns the physical
    flux (consistency of the Godunov flux, Sec. 2.2-2.3)."""
    w, bn = random_states(500, RNG)
    f, cmax = O.riemann(solver, 5.0 / 3.0, w, w, bn)
    for i in range(len(bn)):
        _, fp = O.phys_flux(5.0 / 3.0, w[i], bn[i])
        scale = np.max(np.abs(fp)) + 1.0
        assert np.max(np.abs(f[i] - fp)) <= 1e-13 * scale
        cf = O.fast_speed(5.0 / 3.0, w[i, 0], w[i, 6], bn[i], w[i, 4], w[i, 5])
        assert cmax[i] == pytest.approx(abs(w[i, 1]) + cf, rel=1e-15)


def _hll_conserved(solver_f, ul, ur, fl, fr, sl, sr):
    return (sr * ur - sl * ul - (fr - fl)) / (sr - sl)


@pytest.mark.parametrize("bfield", [True, False])
def test_hll_satisfies_jump_conditions(bfield):
    """HLL (Einfeldt et al. 1991): the single intermediate state is the integral
    average of the Riemann fan, so the flux obeys the Rankine-Hugoniot relation
    across both outer waves."""
    g = 5.0 / 3.0
    w, bn = random_states(300, RNG, bfield)
    wr, _ = random_states(300, RNG, bfield)
    f, _ = O.riemann(O.HLL, g, w, wr, bn)
    for i in range(len(bn)):
        ul, fl = O.phys_flux(g, w[i], bn[i])
        ur, fr = O.phys_flux(g, wr[i], bn[i])
        cl = O.fast_speed(g, w[i, 0], w[i, 6], bn[i], w[i, 4], w[i, 5])
        cr = O.fast_speed(g, wr[i, 0], wr[i, 6], bn[i], wr[i, 4], wr[i, 5])
        sl = min(w[i, 1], wr[i, 1]) - max(cl, cr)
        sr = max(w[i, 1], wr[i, 1]) + max(cl, cr)
        scale = np.max(np.abs(np.concatenate([fl, fr, sl * ul, sr * ur]))) + 1
        if sl >= 0:
            assert np.allclose(f[i], fl, rtol=0, atol=1e-15 * scale)
        elif sr <= 0:
            assert np.allclose(f[i], fr, rtol=0, atol=1e-15 * scale)
        else:
            um = _hll_conserved(None, ul, ur, fl, fr, sl, sr)
            assert np.max(np.abs(f[i] - (fl + sl * (um - ul)))) <= 1e-12 * scale
            assert np.max(np.abs(f[i] - (fr + sr * (um - ur)))) <= 1e-12 * scale


def hllc_reference(g, wl, wr):
    """Test-only HLLC flux for hydrodynamics (Toro 2009, Sec. 10.4), with the same
    outer speed bounds; B = 0.  Face-frame components (rho, mn, mt1, mt2, E)."""
    def parts(w):
        rho, u, v, ww, p = w[0], w[1], w[2], w[3], w[6]
        e = p / (g - 1) + 0.5 * rho * (u * u + v * v + ww * ww)
        U = np.array([rho, rho * u, rho * v, rho * ww, e])
        F = np.array([rho * u, rho * u * u + p, rho * u * v, rho * u * ww, (e + p) * u])
        return U, F, rho, u, v, ww, p, e

    UL, FL, rl, ul, vl, wl_, pl, el = parts(wl)
    UR, FR, rr, ur, vr, wr_, pr, er = parts(wr)
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    sl = min(ul, ur) - max(al, ar)
    sr = max(ul, ur) + max(al, ar)
    if sl >= 0:
        return FL
    if sr <= 0:
        return FR
    ss = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) / (rl * (sl - ul) - rr * (sr - ur))

    def star(U, F, rho, u, v, w, p, e, s):
        fac = rho * (s - u) / (s - ss)
        Us = fac * np.array([1.0, ss, v, w, e / rho + (ss - u) * (ss + p / (rho * (s - u)))])
        return F + s * (Us - U)

    if ss >= 0:
        return star(UL, FL, rl, ul, vl, wl_, pl, el, sl)
    return star(UR, FR, rr, ur, vr, wr_, pr, er, sr)


def test_hlld_without_field_is_hllc():
    """HLLD with B = 0 reduces to the hydrodynamic HLLC solver (Sec. 2.3: HLLC is
    replaced by its magnetised counterpart HLLD)."""
    g = 1.4
    w, bn = random_states(500, RNG, bfield=False)
    wr, _ = random_states(500, RNG, bfield=False)
    f, _ = O.riemann(O.HLLD, g, w, wr, bn)
    for i in range(len(bn)):
        ref = hllc_reference(g, w[i], wr[i])
        scale = np.max(np.abs(ref)) + 1.0
        assert np.max(np.abs(f[i, :5] - ref)) <= 1e-12 * scale
        assert f[i, 5] == 0.0 and f[i, 6] == 0.0


def test_hllc_solver_is_textbook_hllc():
    """The oracle's HLLC (the hydrodynamic solver for B = 0 problems) equals the
    test-only textbook HLLC above, and with B = 0 agrees with HLLD to rounding;
    any field in its input is ignored (no B flux, no magnetic pressure)."""
    g = 5.0 / 3.0
    w, bn = random_states(500, RNG, bfield=False)
    wr, _ = random_states(500, RNG, bfield=False)
    f, cm = O.riemann(O.HLLC, g, w, wr, bn)
    fd, cmd = O.riemann(O.HLLD, g, w, wr, bn)
    for i in range(len(bn)):
        ref = hllc_reference(g, w[i], wr[i])
        scale = np.max(np.abs(ref)) + 1.0
        assert np.max(np.abs(f[i, :5] - ref)) <= 1e-13 * scale
        assert np.max(np.abs(f[i] - fd[i])) <= 1e-12 * scale
        assert f[i, 5] == 0.0 and f[i, 6] == 0.0
    assert np.array_equal(cm, cmd)
    wb, bnb = random_states(50, RNG, bfield=True)
    fb, _ = O.riemann(O.HLLC, g, wb, wb[::-1].copy(), bnb)
    w0 = wb.copy()
    w0[:, 4:6] = 0.0
    f0, _ = O.riemann(O.HLLC, g, w0, w0[::-1].copy(), np.zeros_like(bnb))
    assert np.array_equal(fb, f0)


@pytest.mark.parametrize("bn", [0.0, 0.8, -1.3])
def test_hlld_stationary_contact_and_tangential_discontinuity(bn):
    """Miyoshi & Kusano (2005): HLLD resolves an isolated stationary contact
    (B_n != 0) or tangential discontinuity (B_n = 0) exactly: the flux is the
    physical flux, identical on both sides (no mass flux)."""
    g = 5.0 / 3.0
    if bn != 0.0:  # contact: rho jumps, everything else continuous
        wl = np.array([1.0, 0.0, 0.3, -0.2, 0.5, 0.2, 1.0])
        wr = np.array([0.2, 0.0, 0.3, -0.2, 0.5, 0.2, 1.0])
    else:  # tangential discontinuity: v_t, B_t, rho jump with p_T balanced
        wl = np.array([1.0, 0.0, 0.5, -0.1, 1.0, 0.5, 1.0])
        wr = np.array([0.5, 0.0, -0.3, 0.4, 0.2, 1.1, 1.0])
    f, _ = O.riemann(O.HLLD, g, wl[None], wr[None], np.array([bn]))
    _, fpl = O.phys_flux(g, wl, bn)
    _, fpr = O.phys_flux(g, wr, bn)
    assert np.max(np.abs(fpl - fpr)) <= 1e-15
    assert abs(f[0, 0]) <= 1e-15
    assert np.max(np.abs(f[0] - fpl)) <= 2e-15
    # HLL, by contrast, diffuses the jump: a mass flux appears
    fh, _ = O.riemann(O.HLL, g, wl[None], wr[None], np.array([bn]))
    assert abs(fh[0, 0]) > 1e-3


def rotational_discontinuity(sign_wave, bn, theta=2.0):
    """Left and right face-frame states (rho, vn, vt1, vt2, Bt1, Bt2, p) joined by
    an isolated rotational (Alfven) discontinuity: rho, v_n, p and |B_t| equal on
    both sides, B_t turned by theta, v_t jumping by sign(B_n) dB_t / sqrt(rho)
    for the left-going wave (speed v_n - |B_n|/sqrt(rho)) and by the opposite
    amount for the right-going one (speed v_n + |B_n|/sqrt(rho))."""
    rho, un, p, bt = 1.3, 0.4, 0.8, 0.6
    wl = np.array([rho, un, 0.1, -0.2, bt, 0.0, p])
    wr = wl.copy()
    wr[4:6] = bt * math.cos(theta), bt * math.sin(theta)
    s = math.copysign(1.0, bn)
    dv = sign_wave * s * (wr[4:6] - wl[4:6]) / math.sqrt(rho)
    wr[2:4] = wl[2:4] - dv
    speed = un + sign_wave * abs(bn) / math.sqrt(rho)
    return wl, wr, speed


@pytest.mark.parametrize("sign_wave", [-1, +1])
@pytest.mark.parametrize("bn,un_shift", [(0.9, 0.0), (-0.9, 0.0), (0.9, 0.6), (0.9, -0.7), (-0.5, -0.9)])
def test_hlld_isolated_rotational_discontinuity(sign_wave, bn, un_shift):
    """Miyoshi & Kusano (2005): the HLLD intermediate waves S*_L, S*_R are the
    Alfven waves, so an isolated rotational discontinuity is resolved exactly:
    the flux is the upwind side's physical flux (F_L if the wave moves right of
    the face, F_R if left), which by the Rankine-Hugoniot relation the test
    first checks on the constructed states.  HLL smears it."""
    g = 5.0 / 3.0
    wl, wr, speed = rotational_discontinuity(sign_wave, bn)
    wl[1] += un_shift
    wr[1] += un_shift
    speed += un_shift
    ul, fl = O.phys_flux(g, wl, bn)
    ur, fr = O.phys_flux(g, wr, bn)
    # the states satisfy the jump condition of a discontinuity moving at `speed`
    assert np.max(np.abs((fr - fl) - speed * (ur - ul))) <= 1e-15 * (np.max(np.abs(fl)) + 1)
    assert abs(wl[4] ** 2 + wl[5] ** 2 - wr[4] ** 2 - wr[5] ** 2) <= 1e-15
    f, _ = O.riemann(O.HLLD, g, wl[None], wr[None], np.array([bn]))
    want = fl if speed > 0 else fr
    assert np.max(np.abs(f[0] - want)) <= 4e-15 * (np.max(np.abs(want)) + 1), (f[0], want)
    # HLL does not see the Alfven wave: its flux differs by a finite amount
    fh, _ = O.riemann(O.HLL, g, wl[None], wr[None], np.array([bn]))
    assert np.max(np.abs(fh[0] - want)) > 1e-3


def test_corner_emf_reductions():
    """E^c corner EMF (Gardiner & Stone 2005): (i) for flow along P with no
    Q-variation it returns the Godunov face EMF a1; (ii) for flow along Q with no
    P-variation it returns b1; (iii) with every mass flux zero it is the E^0
    form  (a1+a2+b1+b2)/2 - (c00+c10+c01+c11)/4."""
    for _ in range(200):
        a, b, c0, c1, s = RNG.normal(size=5)
        # (i) 1D along P: a1 = a2 = a; b1 = c10 = c11 = c1; b2 = c00 = c01 = c0; sP = 0
        e = O.corner_emf(a, a, c1, c0, c0, c1, c0, c1, s, s, 0.0, 0.0)
        assert e == pytest.approx(a, abs=4e-16 * (abs(a) + abs(c0) + abs(c1)))
        # (ii) 1D along Q: b1 = b2 = b; a1 = c01 = c11 = c1; a2 = c00 = c10 = c0; sQ = 0
        e = O.corner_emf(c1, c0, b, b, c0, c0, c1, c1, 0.0, 0.0, s, s)
        assert e == pytest.approx(b, abs=4e-16 * (abs(b) + abs(c0) + abs(c1)))
        # (iii) all switches zero
        a1, a2, b1, b2, c00, c10, c01, c11 = RNG.normal(size=8)
        e = O.corner_emf(a1, a2, b1, b2, c00, c10, c01, c11, 0.0, 0.0, 0.0, 0.0)
        e0 = 0.5 * (a1 + a2 + b1 + b2) - 0.25 * (c00 + c10 + c01 + c11)
        assert e == pytest.approx(e0, abs=1e-15 * 8)


def test_corner_emf_picks_upwind_cell():
    """The upwind switch takes the derivative from the cell the mass flux comes
    from: with a positive P-face flux the Q-derivative of row q uses cell p-1."""
    args = dict(a1=0.0, a2=0.0, b1=0.0, b2=0.0, c00=0.0, c10=0.0, c01=1.0, c11=5.0)
    base = [args[k] for k in ("a1", "a2", "b1", "b2", "c00", "c10", "c01", "c11")]
    # only c01 / c11 non-zero: D_Q1 = upw(sq1; c01, c11), D_P3 = upw(sp3; 0, -c01),
    # D_P1 = upw(sp1; 0, -c11)... hold sp at +1 so D_P terms take the first (zero-ish) branch
    e_pos = O.corner_emf(*base, 1.0, 0.0, 1.0, 1.0)
    e_neg = O.corner_emf(*base, -1.0, 0.0, 1.0, 1.0)
    # E = (-D_Q1 + D_P3 - D_P1)/4 with D_P3 = a2 - c00 = 0, D_P1 = c10 - a2 = 0
    assert e_pos == pytest.approx(-1.0 / 4)
    assert e_neg == pytest.approx(-5.0 / 4)


def test_rk_weights_fixture_is_tableau():
    """Tab. weights: each stage's weights sum to 1 (a consistent combination)."""
    w = golden()["rk_weights"]
    for k, v in w.items():
        if k.startswith("_"):
            continue
        for a, b in zip(v["w"], v["w0"]):
            assert a + b == pytest.approx(1.0)
