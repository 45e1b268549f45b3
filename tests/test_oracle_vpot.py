"""Pins of the vector-potential form of constrained transport (Sec. 2.4,
eqs. ind_vec): A on cell edges evolves by dA/dt = -E and B = b0 + curl A.

* The paper states the form is mathematically equivalent to the face-B update:
  both oracle forms agree to round-off over many cycles.
* Its point is that div B does not accumulate round-off: with A it stays at the
  level of a single curl evaluation (no growth with the number of cycles).
* The mean field b0 is carried exactly.
"""
import numpy as np
import pytest

import oracle as O
from paper_2304_13746_amd import inputs as I


def copy_pot(a):
    return {"ax": a["ax"].copy(), "ay": a["ay"].copy(), "az": a["az"].copy(), "b0": a["b0"]}


@pytest.mark.parametrize("integ,emf", [(O.RK2, O.EMF_EC), (O.RK3, O.EMF_EC),
                                       (O.RK2, O.EMF_UCT_HLL), (O.RK2, O.EMF_E0),
                                       (O.RK3, O.EMF_ARITH)])
def test_equivalent_to_face_update(integ, emf):
    n = 16
    s, a = I.orszag_tang_3d(n, potential=True)
    p = O.Params(n, n, n, integrator=integ, emf=emf)
    sa, aa = O.copy_state(s), copy_pot(a)
    O.step_vp(p, sa, aa, 0.0, 0.0, 12)
    sb = O.copy_state(sa)
    # the same start for the face form: the face field b0 + curl A the A form uses
    s0 = O.copy_state(s)
    O.step_vp(p, s0, copy_pot(a), 0.0, 0.0, 0)
    O.step(p, s0, 0.0, 0.0, 12)
    for f in O.FIELDS:
        scale = float(np.max(np.abs(s0[f]))) + 1e-300
        assert float(np.max(np.abs(sa[f] - s0[f]))) <= 1e-11 * max(scale, 1.0), f
    assert not np.array_equal(sb["bx"], s["bx"])


def test_divb_does_not_accumulate():
    n = 16
    s, a = I.orszag_tang_3d(n, potential=True)
    p = O.Params(n, n, n)
    out = {}
    t, dt = 0.0, 0.0
    done = 0
    for k in (5, 200):
        t, dt, _ = O.step_vp(p, s, a, t, dt, k - done)
        done = k
        out[k] = O.diagnostics(p, s)["divb_max"]
    bmax = max(float(np.max(np.abs(s[f]))) for f in ("bx", "by", "bz"))
    assert out[200] / n / bmax <= 1e-14
    assert out[200] <= 4.0 * out[5]
    # the face-B form on the same problem accumulates: larger after 200 cycles
    s2, a2 = I.orszag_tang_3d(n, potential=True)
    O.step_vp(p, s2, a2, 0.0, 0.0, 0)
    O.step(p, s2, 0.0, 0.0, 200)
    assert O.diagnostics(p, s2)["divb_max"] > out[200]


def test_mean_field_is_carried():
    n = 12
    s = I.turbulence(n, seed=2, kpeak=2.0, mach=0.7, b0=(0.2, -0.1, 0.05))
    l = s.pop("_l")
    a = I.uniform_field_potential(s["rho"].shape, (0.2, -0.1, 0.05))
    p = O.Params(n, n, n, *l)
    O.step_vp(p, s, a, 0.0, 0.0, 6)
    d = O.diagnostics(p, s)
    vol = l[0] * l[1] * l[2]
    assert np.allclose(d["bflux"] / vol, [0.2, -0.1, 0.05], rtol=0, atol=1e-15)
    assert np.any(a["az"] != 0.0)
