"""Autotuner on the GPU: tuning leaves the state untouched, picks a timed
shape no slower than the default, and results after tuning are bit-identical
to untuned runs (FP64)."""
import pytest

from gpu_util import bit_equal, need_gpu
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_set_get_launch_roundtrip():
    torch = need_gpu()
    from paper_2304_13746_amd import _lib as L
    from paper_2304_13746_amd.box import MHDBox
    b = MHDBox(24, 16, 40)
    assert b.get_launch()[0] == L.TILE_24x8
    b.set_launch(L.TILE_16x16, 7)
    assert b.get_launch() == (L.TILE_16x16, 7)
    b.set_launch(0, 1000)  # default tile, cap above nz
    assert b.get_launch() == (L.TILE_24x8, 40)
    with pytest.raises(L.MHDError):
        b.set_launch(9, 0)


def test_tune_keeps_state_and_results(tmp_path):
    torch = need_gpu()
    from paper_2304_13746_amd.autotune import Tuner
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox
    spec = I.batch_boxes(5, seed=31, emin=16, emax=64)
    steps = [4, 3, 4, 2, 4]
    stream = torch.cuda.Stream()

    def make():
        out = []
        for sp in spec:
            bx = MHDBox(*sp["dims"], *sp["l"], precision="fp64", stream=stream)
            bx.set_state(sp["state"])
            out.append(bx)
        return out

    ref = make()
    BoxBatch(ref).step(steps)
    ref_out = [b.get_state_numpy() for b in ref]

    tuned = make()
    before = [b.get_state_numpy() for b in tuned]
    batch = BoxBatch(tuned)
    tuner = Tuner(str(tmp_path / "tune.json"), reps=2)
    choice = batch.tune(tuner)
    print("tuned", choice)
    assert not choice["cached"] and choice["candidates"] >= 2
    assert 0.0 < choice["best_ms"] <= choice["default_ms"]
    shapes = {b.get_launch()[0] for b in tuned}
    assert shapes == {choice["tile"]}
    # tuning ran first-stage launches only: state, t and next step unchanged
    for (g0, t0, d0, _), b in zip(before, tuned):
        g1, t1, d1, _ = b.get_state_numpy()
        assert bit_equal(g0, g1) and t0 == t1 and d0 == d1
    batch.step(steps)
    for (e, te, de, _), b in zip(ref_out, tuned):
        g, t, dt, _ = b.get_state_numpy()
        assert bit_equal(e, g) and te == t and de == dt
    # a second tuner on the same cache applies the stored choice without timing
    again = make()
    c2 = BoxBatch(again).tune(Tuner(str(tmp_path / "tune.json")))
    assert c2["cached"] and {b.get_launch()[0] for b in again} == {choice["tile"]}
