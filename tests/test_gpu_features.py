"""GPU tests of the full-size workload, diagnostics, checkpoint/resume, error
latching, launch-shape invariance and determinism (all through the C ABI)."""
import numpy as np
import pytest

import oracle as O
from gpu_util import (FIELDS, bit_equal, check_fp32_cycles, gpu_box, max_rel, need_gpu,
                      run_both)
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def turb256():
    s = I.turbulence(256, seed=2304, kpeak=4.0, mach=0.5, rho0=1.0, p0=0.6, b0=(0.2, 0.0, 0.0))
    s.pop("_l")
    return s


def test_full_size_256_fp64_bit_exact(turb256):
    """The benchmark workload (256^3 turbulence, default launch shape) for one
    RK2 cycle: bit-identical to the oracle, including the next dt."""
    need_gpu()
    g, o, gd, od, (tg, to) = run_both(turb256, (256, 256, 256), 1)
    print("256^3 fp64 max rel", max_rel(g, o))
    assert bit_equal(g, o)
    assert gd == od and tg == to


@pytest.mark.parametrize("opts", [
    {"integrator": "rk3"}, {"recon": "limo3", "integrator": "rk3"},
    {"recon": "ppm", "integrator": "rk3"}, {"emf": "e0"}, {"emf": "arith"}, {"emf": "uct_hll"},
    {"riemann": "hll"}], ids=lambda o: "-".join(o.values()))
def test_full_size_256_options_fp64_bit_exact(turb256, opts):
    """Each scheme option the benchmark times, on the same 256^3 input and in
    the same default launch shape, one cycle: bit-identical to the oracle with
    that option, including the next dt."""
    need_gpu()
    print("256^3 option", opts, flush=True)
    g, o, gd, od, (tg, to) = run_both(turb256, (256, 256, 256), 1, **opts)
    assert bit_equal(g, o)
    assert gd == od and tg == to


def test_full_size_256_vecpot_fp64_bit_exact(turb256):
    """The vector-potential row the benchmark times: the same 256^3 input with its
    uniform field carried as b0 and A = 0, one cycle in the default launch shape:
    state, edge potential and next dt bit-identical to the oracle's potential
    form."""
    need_gpu()
    from paper_2304_13746_amd.box import MHDBox
    pot_f = ("ax", "ay", "az")
    pot = I.uniform_field_potential(turb256["rho"].shape, (0.2, 0.0, 0.0))
    print("256^3 vecpot", flush=True)
    box = MHDBox(256, 256, 256, ct="vecpot", b0=pot["b0"])
    st = dict(turb256)
    st.update({k: pot[k] for k in pot_f})
    box.set_state(st)
    box.step(1)
    g, tg, dg, rc = box.get_state_numpy()
    box.close()
    assert rc == 0
    o = O.copy_state(turb256)
    a = {"ax": pot["ax"].copy(), "ay": pot["ay"].copy(), "az": pot["az"].copy(), "b0": pot["b0"]}
    t, dt, _ = O.step_vp(O.Params(256, 256, 256), o, a, 0.0, 0.0, 1)
    for f in FIELDS:
        assert np.array_equal(g[f], o[f]), f
    for f in pot_f:
        assert np.array_equal(g[f], a[f]), f
    assert tg == t and dg == dt


@pytest.mark.timeout(600)
def test_full_size_256_fp32_ten_cycles(turb256):
    """Ten FP32 cycles at 256^3 from the FP32-rounded input, in the benchmark's
    launch shape: every stage of every cycle against the oracle's stage applied
    to the GPU's own input of that stage, with the GPU's step (density and
    energy element-wise, momentum norm-wise to 1e-5; face fields to 1e-5 plus
    the E^c tie slack of that stage), and each step against eq. (cfl) on the
    GPU state.  The end-to-end difference from the oracle run on the rounded
    input is printed."""
    need_gpu()
    s = I.to_float32_exact(turb256)
    p = O.Params(256, 256, 256)
    box = gpu_box((256, 256, 256), precision="fp32")
    box.set_state(s)
    worst = check_fp32_cycles(box, p, 10)
    g, _, _, _ = box.get_state_numpy()
    box.close()
    o = O.copy_state(s)
    O.step(p, o, 0.0, 0.0, 10)
    print("256^3 fp32, 10 cycles: worst stage errors", worst, "end-to-end max rel", max_rel(g, o))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_diagnostics_match_oracle(precision):
    """Compensated FP64 totals and div B of the GPU state agree with the
    oracle's on the same state to 1e-12 relative; div B stays at round-off."""
    need_gpu()
    s = I.orszag_tang(32)
    if precision == "fp32":
        s = I.to_float32_exact(s)
    box = gpu_box((32, 32, 32), precision=precision)
    box.set_state(s)
    box.step(5)
    g, _, _, _ = box.get_state_numpy()
    d = box.diagnostics()
    ref = O.diagnostics(O.Params(32, 32, 32), g)
    assert d["status"] == 0
    for k in ("mass", "energy"):
        assert abs(d[k] - ref[k]) <= 1e-12 * abs(ref[k])
    vol = 1.0 / 32 ** 3
    for c, f in enumerate(("mx", "my", "mz")):
        assert abs(d["mom"][c] - ref["mom"][c]) <= 1e-12 * np.sum(np.abs(g[f])) * vol
    for c, f in enumerate(("bx", "by", "bz")):
        assert abs(d["bflux"][c] - ref["bflux"][c]) <= 1e-12 * max(np.sum(np.abs(g[f])) * vol, 1e-30)
    assert d["divb_max"] == pytest.approx(ref["divb_max"], rel=1e-12, abs=1e-300)
    assert d["divb_rms"] == pytest.approx(ref["divb_rms"], rel=1e-10, abs=1e-300)
    bmax = max(np.max(np.abs(g[f])) for f in ("bx", "by", "bz"))
    tol = 1e-14 if precision == "fp64" else 1e-6
    assert d["divb_max"] / 32 / bmax <= tol


def test_checkpoint_resume_bit_exact():
    """step(3); get (state, t, dt_next); set into a fresh context; step(4)
    equals step(7) bit for bit."""
    need_gpu()
    s = I.orszag_tang(32)
    a = gpu_box((32, 32, 32))
    a.set_state(s)
    a.step(7)
    ga, ta, da, _ = a.get_state_numpy()
    b = gpu_box((32, 32, 32))
    b.set_state(s)
    b.step(3)
    mid, tm, dm, _ = b.get_state()
    c = gpu_box((32, 32, 32))
    c.set_state(mid, tm, dm)
    c.step(4)
    gc, tc, dc, _ = c.get_state_numpy()
    assert bit_equal(ga, gc) and ta == tc and da == dc


def test_nonphysical_state_is_latched_and_reported():
    """A cell with negative pressure is detected on the device; the next
    synchronising call returns MHD_ERR_NONPHYSICAL; another context is
    unaffected; set_state clears the latch."""
    need_gpu()
    from paper_2304_13746_amd import _lib
    s = I.orszag_tang(16)
    bad = {k: v.copy() for k, v in s.items()}
    bad["en"][3, 5, 7] = 1e-6  # internal energy < 0 there
    good_box = gpu_box((16, 16, 16))
    good_box.set_state(s)
    box = gpu_box((16, 16, 16))
    box.set_state(bad, 0.0, 1e-3)
    box.step(1)
    good_box.step(1)
    _, _, _, rc = box.get_state(check=False)
    assert rc == _lib.MHD_ERR_NONPHYSICAL
    assert box.diagnostics()["status"] == 1
    _, _, _, rc = good_box.get_state(check=False)
    assert rc == _lib.MHD_OK
    box.set_state(s)
    box.step(1)
    _, _, _, rc = box.get_state(check=False)
    assert rc == _lib.MHD_OK


@pytest.mark.parametrize("tile,zchunk", [(1, 16), (1, 7), (2, 32), (2, 3), (3, 0), (3, 5)])
def test_launch_shape_invariance_fp64(tile, zchunk):
    """Tile shape and z-chunk length change only how work is split: FP64
    results are bit-identical to the oracle for every launch shape."""
    need_gpu()
    dims = (40, 36, 28)
    s = I.turbulence(dims, seed=11, kpeak=2.0, mach=0.9, b0=(0.1, 0.3, -0.2))
    s.pop("_l")
    h = 1.0 / 40
    g, o, gd, od, _ = run_both(s, dims, 3, l=(40 * h, 36 * h, 28 * h), tile=tile, zchunk=zchunk)
    assert bit_equal(g, o)
    assert gd == od


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_repeat_runs_identical(precision):
    """Two runs of the same input give identical bits (no races)."""
    need_gpu()
    s = I.orszag_tang_3d(48)
    outs = []
    for _ in range(2):
        box = gpu_box((48, 48, 48), precision=precision)
        box.set_state(s)
        box.step(5)
        outs.append(box.get_state_numpy()[0])
    assert bit_equal(outs[0], outs[1])


def test_t_stop_clips_last_step():
    """With t_stop the cycle that would pass it is shortened to land on it;
    later cycles take zero steps and leave the state unchanged."""
    need_gpu()
    s = I.orszag_tang(16)
    box = gpu_box((16, 16, 16))
    box.set_state(s)
    box.step(3)
    _, t3, dt3, _ = box.get_state()
    t_stop = t3 + 0.5 * dt3
    box.step(1, t_stop=t_stop)
    g1, t4, _, _ = box.get_state_numpy()
    assert t4 == t_stop or abs(t4 - t_stop) <= 1e-15 * t_stop
    box.step(2, t_stop=t_stop)
    g2, t5, _, _ = box.get_state_numpy()
    assert t5 == t4 and bit_equal(g1, g2)


def test_stage_output_availability():
    """mhd_get_stage_output returns the last cycle's stage result only when one
    exists: not before a cycle, not for stages the integrator lacks, not after
    the tuner's timed launches overwrote the buffer; in FP64 stage 1 of an RK2
    cycle is bit-identical to the oracle's Euler stage."""
    need_gpu()
    from paper_2304_13746_amd import _lib as L
    s = I.orszag_tang(16)
    box = gpu_box((16, 16, 16))
    box.set_state(s)
    with pytest.raises(L.MHDError):
        box.get_stage_output(1)
    box.step(1)
    x1 = box.get_stage_output(1)
    _, t, _, _ = box.get_state_numpy()
    with pytest.raises(L.MHDError):
        box.get_stage_output(2)
    want = O.copy_state(s)
    O.step(O.Params(16, 16, 16, integrator=O.EULER), want, 0.0, t, 1)
    assert bit_equal(x1, want)
    import ctypes as C
    arr = (C.c_void_p * 1)(box.ctx.value)
    L.check(box.lib.mhd_tune(arr, 1, 1, None, None), "mhd_tune")
    with pytest.raises(L.MHDError):
        box.get_stage_output(1)
    box.close()
    eul = gpu_box((16, 16, 16), integrator="euler")
    eul.set_state(s)
    eul.step(1)
    with pytest.raises(L.MHDError):
        eul.get_stage_output(1)
    eul.close()
    rk3 = gpu_box((16, 16, 16), integrator="rk3")
    rk3.set_state(s)
    rk3.step(2)
    rk3.get_stage_output(1)
    rk3.get_stage_output(2)
    with pytest.raises(L.MHDError):
        rk3.get_stage_output(3)
    rk3.close()
