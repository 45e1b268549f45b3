"""The vector-potential form of constrained transport on the GPU (Sec. 2.4,
eqs. ind_vec): bit-identical to the oracle's potential form in FP64 (state,
potential and dt sequence), alone and in a batch; FP32 is refused."""
import numpy as np
import pytest

import oracle as O
from gpu_util import FIELDS, bit_equal, need_gpu
from paper_2304_13746_amd import _lib as L
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu
POT = ("ax", "ay", "az")


def copy_pot(a):
    return {"ax": a["ax"].copy(), "ay": a["ay"].copy(), "az": a["az"].copy(), "b0": a["b0"]}


def gpu_run(s, a, dims, l, nsteps, integrator="rk2", riemann="hlld", stream=None, recon="plm",
            emf="ec", **kw):
    from paper_2304_13746_amd.box import MHDBox
    box = MHDBox(*dims, *l, integrator=integrator, riemann=riemann, ct="vecpot", b0=a["b0"],
                 stream=stream, recon=recon, emf=emf, **kw)
    st = dict(s)
    st.update({k: a[k] for k in POT})
    box.set_state(st)
    dts = []
    for _ in range(nsteps):
        box.step(1)
        dts.append(box.get_state()[2])
    g, t, dt, rc = box.get_state_numpy()
    assert rc == 0
    return g, t, dts


@pytest.mark.parametrize("integrator,recon,emf", [("rk2", "plm", "ec"), ("rk3", "plm", "ec"),
                                                  ("rk3", "ppm", "ec"), ("rk2", "plm", "uct_hll"),
                                                  ("rk3", "limo3", "uct_hll"), ("rk2", "plm", "e0"),
                                                  ("rk3", "ppm", "arith")])
@pytest.mark.parametrize("riemann", ["hlld", "hll"])
def test_vecpot_fp64_bit_exact(integrator, riemann, recon, emf):
    need_gpu()
    n = 24
    s, a = I.orszag_tang_3d(n, potential=True)
    dims, l = (n, n, n), (1.0, 1.0, 1.0)
    print("vecpot", integrator, riemann, recon, emf, flush=True)
    g, tg, gd = gpu_run(s, a, dims, l, 5, integrator, riemann, recon=recon, emf=emf)
    o, ao = O.copy_state(s), copy_pot(a)
    p = O.Params(n, n, n, integrator={"rk2": O.RK2, "rk3": O.RK3}[integrator],
                 riemann={"hlld": O.HLLD, "hll": O.HLL}[riemann],
                 recon={"plm": O.PLM, "limo3": O.LIMO3, "ppm": O.PPM}[recon],
                 emf={"ec": O.EMF_EC, "e0": O.EMF_E0, "arith": O.EMF_ARITH,
                      "uct_hll": O.EMF_UCT_HLL}[emf])
    t, dt = 0.0, 0.0
    od = []
    for _ in range(5):
        t, dt, _ = O.step_vp(p, o, ao, t, dt, 1)
        od.append(dt)
    o.update({k: ao[k] for k in POT})
    for f in FIELDS + POT:
        assert np.array_equal(g[f], o[f]), f
    assert gd == od and tg == t


def test_vecpot_mean_field_ragged_batch():
    """Ragged turbulent boxes with a mean field (A = 0 initially, b0 carried):
    a batch equals each box alone, and the first box equals the oracle."""
    torch = need_gpu()
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    specs = []
    for dims, seed in (((40, 24, 18), 3), ((16, 32, 24), 4)):
        s = I.turbulence(dims, seed=seed, kpeak=2.0, mach=0.8, b0=(0.2, -0.1, 0.3))
        l = s.pop("_l")
        specs.append((dims, l, s, I.uniform_field_potential(s["rho"].shape, (0.2, -0.1, 0.3))))
    stream = torch.cuda.Stream()
    boxes = []
    for dims, l, s, a in specs:
        bx = MHDBox(*dims, *l, ct="vecpot", b0=a["b0"], stream=stream)
        st = dict(s)
        st.update({k: a[k] for k in POT})
        bx.set_state(st)
        boxes.append(bx)
    BoxBatch(boxes).step([3, 4])
    for (dims, l, s, a), bx, k in zip(specs, boxes, (3, 4)):
        g, t, dts = gpu_run(s, a, dims, l, k)
        b, tb, _, _ = bx.get_state_numpy()
        assert bit_equal(g, b) and t == tb
        for f in POT:
            assert np.array_equal(g[f], b[f])
    dims, l, s, a = specs[0]
    g, t, _ = gpu_run(s, a, dims, l, 3)
    o, ao = O.copy_state(s), copy_pot(a)
    O.step_vp(O.Params(*dims, *l), o, ao, 0.0, 0.0, 3)
    assert bit_equal(g, o)
    for f in POT:
        assert np.array_equal(g[f], ao[f])


@pytest.mark.parametrize("dims,tile,emf", [((2, 9, 5), L.TILE_24x8, "ec"),
                                           ((1, 1, 33), L.TILE_16x16, "uct_hll"),
                                           ((33, 1, 1), L.TILE_18x11, "e0"),
                                           ((37, 29, 11), L.TILE_18x11, "ec")])
def test_vecpot_narrow_and_ragged_boxes(dims, tile, emf):
    """Extents of one and two cells (the curl and the edge stencils wrap the
    box) and a ragged box, with each tile and short z-chunks, from a seeded
    non-uniform edge potential plus a mean field: state, potential and dt
    sequence bit-identical to the oracle's potential form."""
    need_gpu()
    s = I.turbulence(dims, seed=61, kpeak=1.0, mach=0.7, b0=(0.3, 0.1, 0.2))
    l = s.pop("_l")
    h = l[0] / dims[0]
    rng = np.random.default_rng(61)
    a = {k: 0.05 * h * rng.standard_normal(s["rho"].shape) for k in POT}
    a["b0"] = (0.3, 0.1, 0.2)
    print("vecpot narrow", dims, tile, emf, flush=True)
    g, tg, gd = gpu_run(s, a, dims, l, 3, emf=emf, tile=tile, zchunk=4)
    o, ao = O.copy_state(s), copy_pot(a)
    p = O.Params(*dims, *l, emf={"ec": O.EMF_EC, "e0": O.EMF_E0, "uct_hll": O.EMF_UCT_HLL}[emf])
    t, dt, od = 0.0, 0.0, []
    for _ in range(3):
        t, dt, _ = O.step_vp(p, o, ao, t, dt, 1)
        od.append(dt)
    for f in FIELDS:
        assert np.array_equal(g[f], o[f]), f
    for f in POT:
        assert np.array_equal(g[f], ao[f]), f
    assert gd == od and tg == t


def test_vecpot_fp32_is_refused():
    need_gpu()
    from paper_2304_13746_amd import _lib as L
    from paper_2304_13746_amd.box import MHDBox
    with pytest.raises(L.MHDError):
        MHDBox(16, 16, 16, precision="fp32", ct="vecpot")
