"""UCT-HLLD corner EMFs (Sec. 2.4: the HLLD 2D Riemann solver, after Mignone &
Del Zanna 2021) on the GPU against the FP64 oracle.

The stage kernel exports per-face HLLD coefficients (aL, aR, dL, dR) and the
transverse velocities they weight; two further launches form the edge EMFs and
update the face field (or, with the vector-potential form, feed the potential
update).  FP64 must be bit-identical to the oracle (state and dt sequence);
FP32 is checked stage by stage against the oracle's stage on the GPU's own
stage input (gpu_util.check_fp32_cycles, 1e-5: the coefficients are continuous
in the face states, no E^c-like switch).
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import bit_equal, check_fp32_cycles, gpu_box, max_rel, need_gpu, oracle_params, run_both
from paper_2304_13746_amd import _lib as L
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("recon", ["plm", "limo3", "ppm"])
@pytest.mark.parametrize("integrator", ["rk2", "rk3"])
def test_uct_hlld_fp64_bit_exact(integrator, recon):
    need_gpu()
    dims = (40, 24, 18)
    s = I.turbulence(dims, seed=37, kpeak=2.0, mach=1.0, b0=(0.25, -0.1, 0.2))
    l = s.pop("_l")
    print("uct-hlld", integrator, recon, dims, flush=True)
    g, o, gd, od, (tg, to) = run_both(s, dims, 4, l=l, integrator=integrator, per_step=True,
                                      emf="uct_hlld", recon=recon, zchunk=5)
    print("max rel", max_rel(g, o))
    assert bit_equal(g, o)
    assert gd == od and tg == to


@pytest.mark.parametrize("tile", [L.TILE_16x16, L.TILE_24x8, L.TILE_18x11])
def test_uct_hlld_fp64_every_tile(tile):
    need_gpu()
    dims = (37, 29, 11)
    s = I.turbulence(dims, seed=41, kpeak=2.0, mach=0.9, b0=(0.1, -0.2, 0.25))
    l = s.pop("_l")
    print("uct-hlld tile", tile, flush=True)
    g, o, gd, od, _ = run_both(s, dims, 3, l=l, per_step=True, emf="uct_hlld", tile=tile, zchunk=4)
    assert bit_equal(g, o)
    assert gd == od


@pytest.mark.parametrize("dims", [(2, 9, 5), (1, 1, 33), (33, 1, 1)])
def test_uct_hlld_fp64_narrow_boxes(dims):
    """Extents of one and two cells: the edge stencils wrap the box."""
    need_gpu()
    s = I.turbulence(dims, seed=43, kpeak=1.0, mach=0.7, b0=(0.3, 0.1, 0.2))
    l = s.pop("_l")
    print("uct-hlld narrow", dims, flush=True)
    g, o, gd, od, _ = run_both(s, dims, 3, l=l, per_step=True, emf="uct_hlld", zchunk=2)
    assert bit_equal(g, o)
    assert gd == od


def test_uct_hlld_orszag_tang_fp64():
    need_gpu()
    s = I.orszag_tang(32)
    print("uct-hlld ot fp64", flush=True)
    g, o, _, _, _ = run_both(s, (32, 32, 32), 6, emf="uct_hlld")
    assert bit_equal(g, o)


@pytest.mark.parametrize("recon,integrator", [("plm", "rk2"), ("limo3", "rk3")])
def test_uct_hlld_fp32_every_stage_valid(recon, integrator):
    need_gpu()
    s = I.to_float32_exact(I.orszag_tang(32))
    print("uct-hlld fp32", recon, integrator, flush=True)
    box = gpu_box((32, 32, 32), precision="fp32", emf="uct_hlld", recon=recon, integrator=integrator)
    box.set_state(s)
    p = oracle_params((32, 32, 32), integrator=integrator, emf="uct_hlld", recon=recon)
    worst = check_fp32_cycles(box, p, 5, integrator=integrator)
    box.close()
    print("worst", worst)


def test_uct_hlld_vecpot_fp64_bit_exact():
    """With the vector-potential form the edge EMFs feed the potential update."""
    need_gpu()
    from paper_2304_13746_amd.box import MHDBox
    n = 24
    s, pot = I.orszag_tang(n, potential=True)
    print("uct-hlld vecpot", flush=True)
    box = MHDBox(n, n, n, emf="uct_hlld", ct="vecpot", b0=pot["b0"], integrator="rk3")
    st = dict(s)
    st.update({k: pot[k] for k in ("ax", "ay", "az")})
    box.set_state(st)
    box.step(3)
    g, tg, dg, rc = box.get_state_numpy()
    box.close()
    assert rc == 0
    o = O.copy_state(s)
    a = {"ax": pot["ax"].copy(), "ay": pot["ay"].copy(), "az": pot["az"].copy(), "b0": pot["b0"]}
    t, dt, _ = O.step_vp(O.Params(n, n, n, emf=O.EMF_UCT_HLLD, integrator=O.RK3), o, a, 0.0, 0.0, 3)
    for f in O.FIELDS:
        assert np.array_equal(g[f], o[f]), f
    for f in ("ax", "ay", "az"):
        assert np.array_equal(g[f], a[f]), f
    assert tg == t and dg == dt


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uct_hlld_batch_equals_alone(precision):
    torch = need_gpu()
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    spec = I.batch_boxes(4, seed=91, emin=16, emax=40)
    steps = [3, 2, 4, 3]
    stream = torch.cuda.Stream()
    boxes = []
    print("uct-hlld batch", precision, [sp["dims"] for sp in spec], flush=True)
    for sp in spec:
        bx = MHDBox(*sp["dims"], *sp["l"], precision=precision, emf="uct_hlld", stream=stream)
        bx.set_state(sp["state"])
        boxes.append(bx)
    BoxBatch(boxes).step(steps)
    for sp, n, bx in zip(spec, steps, boxes):
        g, t, dt, _ = bx.get_state_numpy()
        alone = MHDBox(*sp["dims"], *sp["l"], precision=precision, emf="uct_hlld")
        alone.set_state(sp["state"])
        alone.step(n)
        a, ta, da, _ = alone.get_state_numpy()
        assert bit_equal(a, g) and ta == t and da == dt, sp["dims"]


def test_uct_hlld_divb_at_roundoff():
    need_gpu()
    from paper_2304_13746_amd.box import MHDBox
    n = 32
    box = MHDBox(n, n, n, emf="uct_hlld", integrator="rk3")
    box.set_state(I.orszag_tang_3d(n))
    box.step(10)
    d = box.diagnostics()
    g, _, _, _ = box.get_state_numpy()
    box.close()
    bmax = max(float(np.max(np.abs(g[f]))) for f in ("bx", "by", "bz"))
    assert d["divb_max"] / n / bmax <= 1e-14


def test_uct_hlld_full_size_256_fp64_bit_exact():
    """The benchmark's UCT-HLLD row: the 256^3 turbulence input, default launch
    shape, one RK2 cycle, bit-identical to the oracle with the next dt."""
    need_gpu()
    s = I.turbulence(256, seed=2304, kpeak=4.0, mach=0.5, rho0=1.0, p0=0.6, b0=(0.2, 0.0, 0.0))
    s.pop("_l")
    print("uct-hlld 256^3", flush=True)
    g, o, gd, od, (tg, to) = run_both(s, (256, 256, 256), 1, emf="uct_hlld")
    assert bit_equal(g, o)
    assert gd == od and tg == to
