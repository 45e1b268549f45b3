"""Host-side pieces of the FP32 comparisons: the oracle's face mass fluxes and
the E^c upwind-tie slack built from them."""
import numpy as np
import pytest

import oracle as O
from paper_2304_13746_amd import inputs as I


def uniform(n, vx, vy=0.0, vz=0.0, rho=1.0, p=0.6, b=(0.3, 0.2, 0.1)):
    sh = (n, n, n)
    return I.assemble(rho, np.full(sh, vx), np.full(sh, vy), np.full(sh, vz), p,
                      np.full(sh, b[0]), np.full(sh, b[1]), np.full(sh, b[2]), 5.0 / 3.0)


def test_mass_flux_of_uniform_flow_is_rho_v():
    """A uniform state's Riemann mass flux is the physical one, rho v_n."""
    n = 8
    s = uniform(n, 0.3, -0.2, 0.7, rho=1.3)
    fx, fy, fz = O.mass_flux(O.Params(n, n, n), s)
    for a, v in ((fx, 0.3), (fy, -0.2), (fz, 0.7)):
        assert np.allclose(a, 1.3 * v, rtol=1e-14, atol=0)


def test_tie_slack_sits_only_at_near_zero_mass_flux():
    """The face-field slack of a stage is non-zero only next to faces whose mass
    flux lies within the band of zero: none on a turbulent state (no such
    face); on a flow whose v_x crosses zero just off the x-faces 5 and 21 (and
    varies along y, so that the two upwind candidates there differ; v_y and v_z
    keep every y- and z-face flux well away from zero) only on faces within one
    cell of those two slabs."""
    from gpu_util import ec_field_slack
    n = 16
    s = I.turbulence(n, seed=3, kpeak=2.0, mach=0.8, b0=(0.2, 0.0, 0.1))
    l = s.pop("_l")
    p = O.Params(n, n, n, *l)
    sl = ec_field_slack(p, s, 0.3 / O.max_invdt(p, s))
    assert all(np.count_nonzero(sl[f]) == 0 for f in ("bx", "by", "bz"))
    n = 32
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    vx = (0.5 * np.sin(2 * np.pi * (x - 5.0 / n)) + 1e-8) * (1.0 + 0.3 * np.sin(2 * np.pi * y))
    vy = 0.4 + 0.1 * np.cos(2 * np.pi * x)
    sh = (n, n, n)
    s = I.assemble(1.0, vx, vy, np.full(sh, 0.3), 0.6, np.full(sh, 0.3), np.full(sh, 0.2),
                   np.full(sh, 0.1), 5.0 / 3.0)
    p = O.Params(n, n, n)
    fx, _, _ = O.mass_flux(p, s)
    assert abs(fx[0, 0, 5]) < 1e-6 and abs(fx[0, 0, 21]) < 1e-6
    sl = ec_field_slack(p, s, 1e-3)
    cols = set()
    for f in ("bx", "by", "bz"):
        cols |= set(np.unique(np.nonzero(sl[f])[2]).tolist())
    assert {5, 21} <= cols <= {4, 5, 6, 20, 21, 22}
    # the relative band (the default) equals the absolute band it stands for
    band = 1e-5 * max(float(np.max(np.abs(a))) for a in O.mass_flux(p, s))
    sa = ec_field_slack(p, s, 1e-3, band=band)
    assert all(np.array_equal(sa[f], sl[f]) for f in ("bx", "by", "bz"))


def test_tie_spread_bounds_the_e0_difference():
    """E^0 is E^c with every upwind switch at its tie value (the mean of the two
    candidates), so at every edge |E^c - E^0| is at most half of the spread the
    oracle helper reports with every switch counted (band = infinity).  One Euler
    stage with each scheme therefore differs, face by face, by at most the
    face-field bound built from that spread, and the bound is reached within a
    small factor somewhere (it is not vacuous).  A wrong edge or neighbour index
    in the helper or in the bound breaks this."""
    from gpu_util import ec_field_slack
    n = 16
    s = I.turbulence(n, seed=5, kpeak=2.0, mach=0.9, b0=(0.2, -0.1, 0.15))
    l = s.pop("_l")
    dt = 0.3 / O.max_invdt(O.Params(n, n, n, *l), s)
    out = {}
    for emf in (O.EMF_EC, O.EMF_E0):
        p = O.Params(n, n, n, *l, integrator=O.EULER, emf=emf)
        u = O.copy_state(s)
        O.step(p, u, 0.0, dt, 1)
        out[emf] = u
    slack = ec_field_slack(O.Params(n, n, n, *l), s, dt, band=np.inf)
    ratio = 0.0
    for f in ("bx", "by", "bz"):
        d = np.abs(out[O.EMF_EC][f] - out[O.EMF_E0][f])
        assert np.all(d <= 0.5 * slack[f] * (1 + 1e-12) + 1e-15)
        ratio = max(ratio, float(np.max(d / (0.5 * slack[f] + 1e-300))))
    assert ratio > 0.3
    # the fluid is untouched by the corner EMFs within the stage
    for f in ("rho", "mx", "my", "mz", "en"):
        assert np.array_equal(out[O.EMF_EC][f], out[O.EMF_E0][f])


def test_stage_check_accepts_rounding_and_rejects_planted_errors():
    """The stage-wise FP32 check (gpu_util.stage_errors) accepts the oracle's own
    stage rounded to FP32, and the E^0 stage (every switch at its tie value)
    where the slack counts every switch; it rejects a face field moved by 1e-4
    of the largest |B| away from any tie, a density moved by 2e-5 of itself, and
    a stage taken with a 1 % larger step."""
    from gpu_util import assert_stage_valid, ec_field_slack, oracle_stage, stage_errors
    n = 16
    s = I.to_float32_exact(I.orszag_tang(n))
    p = O.Params(n, n, n)
    dt = 0.3 / O.max_invdt(p, s)
    want = oracle_stage(p, s, dt)
    slack = ec_field_slack(p, s, dt)
    got = I.to_float32_exact(want)
    assert_stage_valid(stage_errors(got, want, slack))
    # second stage of RK2, with its weights
    want2 = oracle_stage(p, want, dt, 0.5, 0.5, s)
    assert_stage_valid(stage_errors(I.to_float32_exact(want2), want2, ec_field_slack(p, want, dt, weight=0.5)))
    # E^0 lies within half of the all-switch spread of E^c
    e0 = oracle_stage(O.Params(n, n, n, emf=O.EMF_E0), s, dt)
    assert_stage_valid(stage_errors(e0, want, ec_field_slack(p, s, dt, band=np.inf)))
    bad = O.copy_state(got)
    k = np.unravel_index(np.argmin(slack["by"]), slack["by"].shape)
    assert slack["by"][k] == 0.0
    bad["by"][k] += 1e-4 * max(float(np.max(np.abs(want[f]))) for f in ("bx", "by", "bz"))
    with pytest.raises(AssertionError):
        assert_stage_valid(stage_errors(bad, want, slack))
    bad = O.copy_state(got)
    bad["rho"][3, 4, 5] *= 1 + 2e-5
    with pytest.raises(AssertionError):
        assert_stage_valid(stage_errors(bad, want, slack))
    with pytest.raises(AssertionError):
        assert_stage_valid(stage_errors(oracle_stage(p, s, dt * (1 + 1e-2)), want, slack))


def test_switch_changes_reproduce_e0():
    """E^0 is E^c with every upwind switch at the mean of its two candidates.
    The face-field changes gpu_util.ec_switch_changes derives for that choice
    at every switch (listed by oracle.ec_ties with an unbounded band), added to
    the E^c stage, give the oracle's E^0 stage to rounding, while the two
    stages themselves differ by about 1e-2: the switch list, the slot signs, the
    edge stencil and the Stokes coefficients are all as the stage applies them."""
    import dataclasses

    from gpu_util import ec_switch_changes, oracle_stage
    n = 16
    s = I.turbulence((n, n, n), seed=3, kpeak=2.0, mach=0.8, b0=(0.2, 0.1, -0.1))
    l = s.pop("_l")
    p = O.Params(n, n, n, *l)
    dt = p.cfl / O.max_invdt(p, s)
    for w in (1.0, 0.5):
        ec = oracle_stage(p, s, dt, w, 1.0 - w, s)
        e0 = oracle_stage(dataclasses.replace(p, emf=O.EMF_E0), s, dt, w, 1.0 - w, s)
        ties = O.ec_ties(p, s, 1e300)
        assert len(ties[0]) == 12 * n ** 3
        acc = {f: ec[f].copy().ravel() for f in ("bx", "by", "bz")}
        for per_alt in ec_switch_changes(p, ties, dt, w, alternatives="mean"):
            for comp, c, v in per_alt[0]:
                acc[comp][c] += v
        for f in ("bx", "by", "bz"):
            sc = float(np.max(np.abs(e0[f])))
            assert np.max(np.abs(acc[f].reshape(e0[f].shape) - e0[f])) <= 1e-14 * sc
            assert np.max(np.abs(ec[f] - e0[f])) >= 1e-3 * sc


def _crossing_state(n=32):
    """v_x crosses zero just off the x-faces 5 and 21, where v_y jumps from -0.4
    to 0.4 (a shear layer); B_x varies along y only (divergence-free), so the
    y-derivatives of E_z that the x-face switches pick between differ by about
    0.8 dB_x/dy on the two sides, while pressure and the other field components
    are uniform and the faces' mass flux stays within 1e-7 of zero."""
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    vx = (0.5 * np.sin(2 * np.pi * (x - 5.0 / n)) + 1e-8) * (1.0 + 0.3 * np.sin(2 * np.pi * y))
    vy = np.where((x > 5.0 / n) & (x < 21.0 / n), 0.4, -0.4)
    bx = 0.3 + 0.2 * np.sin(2 * np.pi * y)
    sh = (n, n, n)
    return I.to_float32_exact(I.assemble(1.0, vx, vy, np.full(sh, 0.3), 0.6, bx,
                                         np.full(sh, 0.2), np.full(sh, 0.1), 5.0 / 3.0))


def test_exact_tie_check_explains_other_choices_and_rejects_the_rest():
    """A stage result in which some switches at near-zero mass flux take another
    candidate (rounded to FP32) passes the E^c check with every departing face
    explained; the same result with a face moved by 1e-4 of max |B| away from any
    tie, or with a tie face moved by a quarter of what the other candidate gives
    (neither it nor the mean of the two), fails."""
    from gpu_util import check_fp32_stage, ec_switch_changes, oracle_stage
    n = 32
    s = _crossing_state(n)
    p = O.Params(n, n, n)
    dt = p.cfl / O.max_invdt(p, s)
    want = oracle_stage(p, s, dt)
    ties = O.ec_ties(p, s, -1e-5)
    assert 0 < len(ties[0]) < 12 * n ** 3 // 10
    changes = ec_switch_changes(p, ties, dt)
    bsc = max(float(np.max(np.abs(want[f]))) for f in ("bx", "by", "bz"))
    # the switches whose other candidate moves a face by more than 1e-5
    big = [q for q, per_alt in enumerate(changes) if max(abs(v) for _, _, v in per_alt[0]) > 3e-5 * bsc]
    assert len(big) >= 4
    got = {f: v.copy() for f, v in want.items()}
    flat = {f: got[f].reshape(-1) for f in ("bx", "by", "bz")}
    for q in big[::7][:6]:
        for comp, c, v in changes[q][0]:
            flat[comp][c] += v
    got = I.to_float32_exact(got)
    e = check_fp32_stage(p, s, dt, got)
    assert e["b_bad"] > 0 and e["b_unexplained"] == 0, e
    # a departure where no switch reaches
    tie_cells = {c for per_alt in changes for ch in per_alt for _, c, _ in ch}
    far = next(c for c in range(n ** 3) if c not in tie_cells)
    bad = {f: v.copy() for f, v in got.items()}
    bad["by"].reshape(-1)[far] += 1e-4 * bsc
    with pytest.raises(AssertionError):
        check_fp32_stage(p, s, dt, bad)
    # a tie face moved by a quarter of what the other candidate gives (the mean
    # of the two gives half)
    comp, c, v = max((ch for q in big for ch in changes[q][0]), key=lambda ch: abs(ch[2]))
    assert abs(v) > 1e-4 * bsc
    part = {f: v2.copy() for f, v2 in want.items()}
    part[comp].reshape(-1)[c] += 0.25 * v
    with pytest.raises(AssertionError):
        check_fp32_stage(p, s, dt, I.to_float32_exact(part))
