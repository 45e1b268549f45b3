"""Host logic of the launch-shape autotuner: cache keys, cache hits, corrupt
cache files (the timing itself runs on the GPU in test_gpu_autotune.py)."""
import json
import types

import pytest

from paper_2304_13746_amd import _lib as L
from paper_2304_13746_amd.autotune import Tuner, group_key


class FakeBox:
    def __init__(self, nx, ny, nz, precision="fp32"):
        self.shape = (nz, ny, nx)
        self.precision = precision
        self.params = types.SimpleNamespace(riemann=L.MHD_HLLD, recon=L.MHD_PLM,
                                            emf=L.MHD_EMF_EC)
        self.launch = None

    def set_launch(self, tile, zchunk):
        self.launch = (tile, zchunk)


def fake_tuner(tmp_path, monkeypatch, result):
    calls = []
    monkeypatch.setattr(Tuner, "_device_name", staticmethod(lambda box: "gfx950-test"))

    def measure(self, boxes, stream=None):
        calls.append([b.shape for b in boxes])
        for b in boxes:
            b.set_launch(result["tile"], result["zchunk_cap"])
        return dict(result)

    monkeypatch.setattr(Tuner, "measure", measure)
    return Tuner(str(tmp_path / "tune.json")), calls


def test_group_key_ignores_order_and_separates_groups():
    a = group_key("d", "fp32", "hlld", [(16, 16, 16), (32, 24, 8)])
    b = group_key("d", "fp32", "hlld", [(32, 24, 8), (16, 16, 16)])
    assert a == b
    assert a != group_key("d", "fp64", "hlld", [(16, 16, 16), (32, 24, 8)])
    assert a != group_key("d", "fp32", "hll", [(16, 16, 16), (32, 24, 8)])
    assert a != group_key("d", "fp32", "hlld", [(16, 16, 16), (24, 32, 8)])


def test_measure_once_then_cache_hit(tmp_path, monkeypatch):
    res = {"tile": L.TILE_16x16, "zchunk_cap": 32, "best_ms": 1.0, "default_ms": 1.5,
           "candidates": 12}
    tuner, calls = fake_tuner(tmp_path, monkeypatch, res)
    boxes = [FakeBox(16, 16, 16), FakeBox(40, 24, 64)]
    c1 = tuner.tune(boxes)
    assert not c1["cached"] and len(calls) == 1
    # a new tuner reads the file; the same group in another order is a hit
    tuner2 = Tuner(str(tmp_path / "tune.json"))
    boxes2 = [FakeBox(40, 24, 64), FakeBox(16, 16, 16)]
    c2 = tuner2.tune(boxes2)
    assert c2["cached"] and len(calls) == 1
    assert all(b.launch == (L.TILE_16x16, 32) for b in boxes2)
    # force re-measures
    tuner2.tune(boxes2, force=True)
    assert len(calls) == 2
    data = json.load(open(tmp_path / "tune.json"))
    assert len(data) == 1


@pytest.mark.parametrize("content", ["", "not json", "[1, 2]"])
def test_corrupt_cache_is_ignored(tmp_path, monkeypatch, content):
    (tmp_path / "tune.json").write_text(content)
    res = {"tile": L.TILE_24x8, "zchunk_cap": 0, "best_ms": 1.0, "default_ms": 1.0,
           "candidates": 6}
    tuner, calls = fake_tuner(tmp_path, monkeypatch, res)
    c = tuner.tune([FakeBox(64, 64, 64)])
    assert not c["cached"] and len(calls) == 1
    assert json.load(open(tmp_path / "tune.json"))


def test_cached_per_class_zchunks_are_applied(tmp_path, monkeypatch):
    """A cached choice with per-class z-chunks (boxes sharing nz) gives each box
    its class's value, and the common cap to a class the entry does not name."""
    res = {"tile": L.TILE_24x8, "zchunk_cap": 16, "best_ms": 1.0, "default_ms": 1.2,
           "candidates": 20, "zchunk_by_nz": {"64": 32, "16": 16}}
    tuner, calls = fake_tuner(tmp_path, monkeypatch, res)
    boxes = [FakeBox(16, 16, 16), FakeBox(40, 24, 64), FakeBox(8, 8, 64)]
    tuner.tune(boxes)
    tuner2 = Tuner(str(tmp_path / "tune.json"))
    boxes2 = [FakeBox(8, 8, 64), FakeBox(16, 16, 16), FakeBox(40, 24, 64)]
    c = tuner2.tune(boxes2)
    assert c["cached"] and len(calls) == 1
    assert [b.launch for b in boxes2] == [(L.TILE_24x8, 32), (L.TILE_24x8, 16), (L.TILE_24x8, 32)]
    other = FakeBox(8, 8, 48)
    tuner2.apply([other], c)
    assert other.launch == (L.TILE_24x8, 16)
