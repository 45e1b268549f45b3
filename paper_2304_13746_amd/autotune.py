"""Launch-shape autotuner with a persistent cache.

``mhd_tune`` (libmhd) times the first-stage launch of a group of boxes, as one
batched launch, for every stage-kernel tile and z-chunk cap, takes the fastest
common shape and then refines the z-chunk per shape class (boxes sharing nz).
This module keys that choice by the GPU, the precision,
the scheme (solver, reconstruction, EMF) and the multiset of box shapes, keeps
it in a JSON file, and applies a cached choice on later calls without timing
anything.  The launch shape only
changes how the work is split, never the result (FP64 is bit-identical for
every shape), so a stale cache entry can cost time but not correctness.

    tuner = Tuner()                 # cache in $MHD_TUNE_CACHE or ~/.cache
    choice = tuner.tune(boxes)      # {"tile": 2, "zchunk_cap": 32, ...}
"""
from __future__ import annotations

import ctypes as C
import json
import os
import threading

from . import _lib as L

TILE_NAMES = {L.TILE_16x16: "16x16", L.TILE_24x8: "24x8", L.TILE_18x11: "18x11"}


def default_cache_path() -> str:
    env = os.environ.get("MHD_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2304_13746_amd", "tune.json")


def group_key(device_name: str, precision: str, scheme: str, shapes) -> str:
    """Cache key: device, precision, scheme and the sorted (nx, ny, nz) list."""
    dims = sorted(tuple(int(v) for v in s) for s in shapes)
    return json.dumps([device_name, precision, scheme, dims], separators=(",", ":"))


class Tuner:
    """Chooses and applies launch shapes for groups of MHDBox objects."""

    def __init__(self, path: str | None = None, reps: int = 3):
        self.path = path or default_cache_path()
        self.reps = int(reps)
        self._lock = threading.Lock()
        self._cache = self._load()

    def _load(self) -> dict:
        try:
            with open(self.path) as fh:
                data = json.load(fh)
            return data if isinstance(data, dict) else {}
        except (OSError, ValueError):
            return {}

    def _save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(self._cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    @staticmethod
    def _device_name(box) -> str:
        import torch
        p = torch.cuda.get_device_properties(box.device)
        return f"{p.name}/{getattr(p, 'gcnArchName', '')}"

    def key(self, boxes) -> str:
        b0 = boxes[0]
        pr = b0.params
        scheme = f"riemann{pr.riemann}/recon{pr.recon}/emf{pr.emf}"
        return group_key(self._device_name(b0), b0.precision, scheme,
                         [(b.shape[2], b.shape[1], b.shape[0]) for b in boxes])

    def lookup(self, boxes):
        return self._cache.get(self.key(boxes))

    def apply(self, boxes, choice: dict):
        per_nz = choice.get("zchunk_by_nz", {})
        for b in boxes:
            b.set_launch(choice["tile"], per_nz.get(str(b.shape[0]), choice["zchunk_cap"]))

    def measure(self, boxes, stream=None) -> dict:
        """Time every candidate on the GPU (mhd_tune) and apply the fastest."""
        lib = boxes[0].lib
        arr = (C.c_void_p * len(boxes))(*[b.ctx.value for b in boxes])
        res = L.TuneResult()
        st = stream if stream is not None else boxes[0].stream
        L.check(lib.mhd_tune(arr, len(boxes), self.reps, C.c_void_p(st.cuda_stream), C.byref(res)),
                "mhd_tune")
        # the z-planes per work-group each shape class ended with
        per_nz = {str(b.shape[0]): b.get_launch()[1] for b in boxes}
        return {"tile": res.tile, "zchunk_cap": res.zchunk_cap, "best_ms": res.best_ms,
                "default_ms": res.default_ms, "candidates": res.candidates,
                "zchunk_by_nz": per_nz}

    def tune(self, boxes, stream=None, force: bool = False) -> dict:
        """Apply the cached shape for this group, or measure, store and apply."""
        if not boxes:
            raise ValueError("no boxes to tune")
        key = self.key(boxes)
        with self._lock:
            hit = None if force else self._cache.get(key)
            if hit is not None:
                self.apply(boxes, hit)
                return dict(hit, cached=True)
            choice = self.measure(boxes, stream)
            self._cache[key] = choice
            self._save()
        return dict(choice, cached=False)
