"""Batched launches: each box is bit-identical alone and in a batch of uneven
boxes (FP32 and FP64), and a captured HIP graph replays the eager result."""
import numpy as np
import pytest

from gpu_util import FIELDS, bit_equal, need_gpu
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu


def small_batch(n=6, seed=77):
    boxes = I.batch_boxes(n, seed=seed, emin=16, emax=48)
    return boxes


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_alone(precision):
    torch = need_gpu()
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    spec = small_batch()
    steps = [3, 5, 4, 5, 2, 5]
    stream = torch.cuda.Stream()
    boxes = []
    for b, sp in enumerate(spec):
        bx = MHDBox(*sp["dims"], *sp["l"], precision=precision, stream=stream)
        bx.set_state(sp["state"])
        boxes.append(bx)
    BoxBatch(boxes).step(steps)
    mixed = [bx.get_state_numpy() for bx in boxes]
    for sp, n, (g, t, dt, _) in zip(spec, steps, mixed):
        alone = MHDBox(*sp["dims"], *sp["l"], precision=precision)
        alone.set_state(sp["state"])
        alone.step(n)
        a, ta, da, _ = alone.get_state_numpy()
        assert bit_equal(a, g) and ta == t and da == dt, sp["dims"]


def test_graph_replay_matches_eager():
    """Capture 3 cycles of a 4-box FP32 batch; replay it three times with
    eager work and synchronisation in between; after every replay the state
    equals an eager run of the same total cycle count."""
    torch = need_gpu()
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    spec = small_batch(4, seed=5)
    stream = torch.cuda.Stream()
    gb = []
    for sp in spec:
        bx = MHDBox(*sp["dims"], *sp["l"], precision="fp32", stream=stream)
        bx.set_state(sp["state"])
        gb.append(bx)
    batch = BoxBatch(gb)
    graph = batch.capture(3)
    torch.cuda.synchronize()
    # capture does not execute: the states are still the initial ones
    for sp, bx in zip(spec, gb):
        g, t, _, _ = bx.get_state_numpy()
        assert t == 0.0
    ref = []
    for sp in spec:
        bx = MHDBox(*sp["dims"], *sp["l"], precision="fp32")
        bx.set_state(sp["state"])
        ref.append(bx)
    for rep in range(1, 4):
        graph.replay()
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work
        for bx in ref:
            bx.step(3)
        for bx, r in zip(gb, ref):
            g, t, dt, _ = bx.get_state_numpy()
            e, te, de, _ = r.get_state_numpy()
            assert bit_equal(g, e) and t == te and dt == de, rep


def test_rk3_batch_and_graph_match_alone():
    """RK3 boxes: a batch equals each box alone, and a captured graph replays
    the eager result (FP64, bit for bit)."""
    torch = need_gpu()
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    spec = small_batch(4, seed=9)
    stream = torch.cuda.Stream()
    boxes = []
    for sp in spec:
        bx = MHDBox(*sp["dims"], *sp["l"], integrator="rk3", stream=stream)
        bx.set_state(sp["state"])
        boxes.append(bx)
    graph = BoxBatch(boxes).capture(2)
    for _ in range(2):
        graph.replay()
        torch.cuda.synchronize()
    for sp, bx in zip(spec, boxes):
        alone = MHDBox(*sp["dims"], *sp["l"], integrator="rk3")
        alone.set_state(sp["state"])
        alone.step(4)
        a, ta, da, _ = alone.get_state_numpy()
        g, t, dt, _ = bx.get_state_numpy()
        assert bit_equal(a, g) and ta == t and da == dt, sp["dims"]


def test_batch_of_mixed_physics_matches_oracle():
    """One batched launch per stage over boxes that differ in every per-box
    parameter the batch allows to differ: extents, domain lengths (so cell
    widths), adiabatic index, CFL number and step count.  Each box's state,
    time and next step are bit-identical to the oracle run alone with that
    box's own parameters (a descriptor or scalar taken from the wrong box
    would show here)."""
    torch = need_gpu()
    import oracle as O
    from gpu_util import oracle_params
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    cases = [((20, 33, 17), (1.0, 1.5, 0.8), 5.0 / 3.0, 0.3, 3, 81),
             ((40, 16, 24), (2.0, 1.0, 1.0), 1.4, 0.5, 4, 83),
             ((24, 24, 9), (1.0, 1.0, 1.0), 2.0, 0.2, 2, 85)]
    stream = torch.cuda.Stream()
    boxes, states = [], []
    for dims, l, gamma, cfl, _, seed in cases:
        s = I.turbulence(dims, seed=seed, kpeak=2.0, mach=1.0, b0=(0.2, 0.1, -0.1), gamma=gamma, l=l)
        s.pop("_l")
        bx = MHDBox(*dims, *l, gamma=gamma, cfl=cfl, stream=stream)
        bx.set_state(s)
        boxes.append(bx)
        states.append(s)
    print("mixed batch", [c[:5] for c in cases], flush=True)
    BoxBatch(boxes).step([c[4] for c in cases])
    for (dims, l, gamma, cfl, n, _), bx, s in zip(cases, boxes, states):
        g, tg, dg, rc = bx.get_state_numpy()
        bx.close()
        p = oracle_params(dims, l, gamma=gamma, cfl=cfl)
        o = O.copy_state(s)
        t, dt, _ = O.step(p, o, 0.0, 0.0, n)
        assert rc == 0
        assert bit_equal(g, o) and tg == t and dg == dt, dims


@pytest.mark.parametrize("riemann,recon,integrator", [("hlld", "ppm", "rk3"),
                                                      ("hllc", "ppm", "rk2"),
                                                      ("hllc", "limo3", "rk3")])
def test_batch_of_option_builds_matches_oracle(riemann, recon, integrator):
    """Batched launches of the option builds with their own LDS layouts and
    halos: PPM (three-cell halo, five-plane z-window) with HLLD, and the
    field-free HLLC build with PPM and with LimO3; three uneven boxes with
    their own step counts, each bit-identical to the oracle run alone."""
    torch = need_gpu()
    import oracle as O
    from gpu_util import oracle_params
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    b0 = (0.0, 0.0, 0.0) if riemann == "hllc" else (0.2, -0.1, 0.1)
    cases = [((26, 19, 21), 3, 91), ((16, 40, 12), 2, 93), ((33, 24, 30), 3, 95)]
    stream = torch.cuda.Stream()
    boxes, states, lens = [], [], []
    for dims, _, seed in cases:
        s = I.turbulence(dims, seed=seed, kpeak=2.0, mach=1.2, b0=b0)
        l = s.pop("_l")
        bx = MHDBox(*dims, *l, riemann=riemann, recon=recon, integrator=integrator, stream=stream)
        bx.set_state(s)
        boxes.append(bx)
        states.append(s)
        lens.append(l)
    print("option batch", riemann, recon, integrator, [c[0] for c in cases], flush=True)
    BoxBatch(boxes).step([c[1] for c in cases])
    for (dims, n, _), bx, s, l in zip(cases, boxes, states, lens):
        g, tg, dg, rc = bx.get_state_numpy()
        bx.close()
        p = oracle_params(dims, l, riemann, integrator, recon=recon)
        o = O.copy_state(s)
        t, dt, _ = O.step(p, o, 0.0, 0.0, n)
        assert rc == 0
        assert bit_equal(g, o) and tg == t and dg == dt, dims
