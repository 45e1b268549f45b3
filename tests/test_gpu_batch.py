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
