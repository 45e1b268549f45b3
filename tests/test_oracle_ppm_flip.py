"""The oracle's PPM decision hook (reading R21) and the FP32 PPM stage check
built on it (gpu_util.ppm_flip_check), on the CPU.

Three PPM decisions make a face value jump when they change (Sec. 2.3; Colella
& Woodward 1984, Colella & Sekora 2008): an interface value outside the interval
of its two cells, a cell at an extremum, D2 = 0.  The hook takes chosen near
decisions the other way; what it must reproduce is the result that an input
moved across the threshold gives, since that is what a lower-precision
evaluation rounding the test the other way produces.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import STAGE_WEIGHTS, oracle_params, oracle_stage, ppm_flip_check
from paper_2304_13746_amd import inputs as I

BAND = 1e-6
DELTA = 1e-9  # distance of a constructed test from its threshold (relative 1e-9 < BAND)


@pytest.fixture(autouse=True)
def _hook_off():
    yield
    O.set_ppm_flip(0.0)


def _near_count(a):
    O.set_ppm_flip(BAND, 1 << 60)
    O.ppm_faces(a)
    n = O.ppm_flips()
    O.set_ppm_flip(0.0)
    return n


def _flipped(a, target=0):
    O.set_ppm_flip(BAND, target)
    r = O.ppm_faces(a)
    O.set_ppm_flip(0.0)
    return r


def _across(kind, rng):
    """A stencil whose one near decision is `kind`, and the same stencil with the
    tested quantity moved to the other side of the threshold."""
    a = rng.uniform(0.0, 2.0, 5)
    if kind == "extremum":  # a_{j-1} just below a_j (or a_{j+1} just above)
        if rng.random() < 0.5:
            a[1] = a[2] - DELTA
            b = a.copy()
            b[1] = a[2] + DELTA
        else:
            a[3] = a[2] + DELTA
            b = a.copy()
            b[3] = a[2] - DELTA
        return a, b
    # the upper interface value of cell j sits DELTA above a_j:
    # 7/12 (a_j + a_{j+1}) - 1/12 (a_{j-1} + a_{j+2}) = a_j + s DELTA
    def mk(s):
        c = a.copy()
        c[4] = 7.0 * (c[2] + c[3]) - c[1] - 12.0 * (c[2] + s * DELTA)
        return c
    return mk(1.0), mk(-1.0)


@pytest.mark.parametrize("kind", ["extremum", "interface"])
def test_flip_equals_input_moved_across_threshold(kind):
    """Where exactly one decision is near, taking it the other way gives what the
    input moved across its threshold gives (to the size of the move), and in
    many such stencils that is far from the unflipped result: the decision
    jumps."""
    rng = np.random.default_rng(2304 if kind == "extremum" else 2305)
    single, jumped = 0, 0
    for _ in range(600):
        a, b = _across(kind, rng)
        if _near_count(a) != 1:
            continue
        single += 1
        base, moved, fl = O.ppm_faces(a), O.ppm_faces(b), _flipped(a)
        assert max(abs(fl[0] - moved[0]), abs(fl[1] - moved[1])) <= 1e-7, (a, base, fl, moved)
        if max(abs(base[0] - moved[0]), abs(base[1] - moved[1])) > 1e-3:
            jumped += 1
    assert single >= 200 and jumped >= 100, (single, jumped)


def test_equal_and_far_values_are_not_near():
    """Equal neighbouring values are equal in any precision, and decisions far
    from their thresholds are not near: no count, and the hook changes nothing."""
    rng = np.random.default_rng(11)
    for a in ([1.0] * 5, [0.3, 0.7, 0.7, 0.7, 0.2], [2.0, 1.0, 1.0, 3.0, 0.5]):
        assert _near_count(np.array(a)) == 0
        assert _flipped(np.array(a)) == O.ppm_faces(np.array(a))
    for _ in range(200):
        a = np.cumsum(rng.uniform(0.1, 1.0, 5))  # strictly monotone, well separated
        if _near_count(a) == 0:
            assert _flipped(a) == O.ppm_faces(a)


def _stage_input(n=16):
    """The Sedov blast after two RK3 cycles, rounded to FP32 after each (as an
    FP32 run holds it): the blast front has cells whose values differ by an
    FP32 ulp, where PPM decisions sit near their thresholds."""
    s = I.to_float32_exact(I.sedov(n))
    p = oracle_params((n, n, n), riemann="hllc", integrator="rk3", recon="ppm")
    t, dt = 0.0, 0.0
    for _ in range(2):
        t, dt, _ = O.step(p, s, t, dt, 1)
        s = I.to_float32_exact(s)
    pe = oracle_params((n, n, n), riemann="hllc", integrator="euler", recon="ppm")
    return pe, s, dt


def test_hook_off_is_the_method_and_picks_match_targets():
    p, x, dt = _stage_input()
    ref = oracle_stage(p, x, dt)
    O.set_ppm_flip(BAND, 1 << 60)
    oracle_stage(p, x, dt)
    sites = O.ppm_sites()
    assert len(sites) == O.ppm_flips() > 0
    O.set_ppm_flip(0.0)
    again = oracle_stage(p, x, dt)
    assert all(np.array_equal(ref[f], again[f]) for f in O.FIELDS)
    start = np.r_[0, np.flatnonzero(np.diff(sites) != 0) + 1]
    ords = np.arange(len(sites)) - np.repeat(start, np.diff(np.r_[start, len(sites)]))
    ncell = x["rho"].size
    for t in np.linspace(0, len(sites) - 1, 5).astype(int):
        O.set_ppm_flip(BAND, int(t))
        by_target = oracle_stage(p, x, dt)
        O.set_ppm_flip(BAND, 1 << 60)
        O.set_ppm_pick(sites[t:t + 1], ords[t:t + 1], 4 * ncell)
        by_pick = oracle_stage(p, x, dt)
        assert all(np.array_equal(by_target[f], by_pick[f]) for f in O.FIELDS), t
    O.set_ppm_flip(0.0)


def test_stage_check_explains_flips_and_catches_other_departures():
    """A stage result that takes some near decisions the other way (and is
    rounded to FP32) passes the check with every departing cell explained; the
    same result with one cell moved by 1e-4 fails it."""
    p, x, dt = _stage_input()
    base = oracle_stage(p, x, dt)
    O.set_ppm_flip(BAND, 1 << 60)
    oracle_stage(p, x, dt)
    sites = O.ppm_sites()
    start = np.r_[0, np.flatnonzero(np.diff(sites) != 0) + 1]
    ords = np.arange(len(sites)) - np.repeat(start, np.diff(np.r_[start, len(sites)]))
    # near decisions whose flip moves some cell by more than 1e-5
    strong = []
    for t in range(0, len(sites), max(1, len(sites) // 60)):
        O.set_ppm_flip(BAND, t)
        alt = oracle_stage(p, x, dt)
        if np.max(np.abs(alt["rho"] - base["rho"]) / base["rho"]) > 1e-4:
            strong.append(t)
        if len(strong) == 3:
            break
    O.set_ppm_flip(0.0)
    assert strong, "no near decision of consequence in this input"
    # take them the other way together (distinct sites), then round to FP32
    keep = {}
    for t in strong:
        keep.setdefault(int(sites[t]), int(ords[t]))
    O.set_ppm_flip(BAND, 1 << 60)
    O.set_ppm_pick(list(keep), list(keep.values()), 4 * x["rho"].size)
    got = oracle_stage(p, x, dt)
    O.set_ppm_flip(0.0)
    got = {f: v.astype(np.float32).astype(np.float64) for f, v in got.items()}
    r = ppm_flip_check(p, x, dt, got)
    assert r["bad"] > 0 and r["unexplained"] == 0, r
    # a departure no decision explains
    quiet = np.argwhere(np.abs(got["rho"] - base["rho"]) <= 1e-7 * base["rho"])[0]
    bad = {f: v.copy() for f, v in got.items()}
    bad["rho"][tuple(quiet)] *= 1.0 + 1e-4
    r = ppm_flip_check(p, x, dt, bad)
    assert r["unexplained"] >= 1, r
