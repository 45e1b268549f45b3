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
