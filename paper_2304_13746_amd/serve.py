"""Continuous-batching server for MHD box requests.

Requests (box edge, step count, initial condition) arrive over time.  The
server admits a queued request when its workspace fits the HBM budget and a slot
is free (first come first served, with a bounded skip-ahead so one large box does
not block small ones behind it), keeps every admitted box resident in HBM, and
advances all admitted boxes together in epochs of batched launches
(``mhd_step_batch``).  Boxes admitted while others run join the next epoch;
finished boxes retire (state copied out, workspace freed) and make room for the
next admissions.  Two epochs are kept in flight so the GPU never idles while the
host admits and retires.  Latency of a request = completion - arrival.

The scheduling logic is backend-agnostic; ``GpuBackend`` drives libmhd through
MHDBox / BoxBatch, and tests drive the same ``Server`` with a virtual-time mock.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

EDGES = (32, 48, 64, 96, 128, 192)


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the replay
    edge: int
    steps: int
    init: str  # "ot" (Orszag-Tang) or "turb" (turbulence)
    seed: int


@dataclass
class Done:
    rid: int
    arrival: float
    admitted: float
    finished: float
    cells: int
    steps: int
    status: int
    result: object = None

    @property
    def latency(self):
        return self.finished - self.arrival


def poisson_requests(n: int, rate: float, seed: int = 2304, edges=EDGES, steps=(10, 200)):
    """n requests with exponential inter-arrival gaps (mean 1/rate), edge uniform
    in ``edges``, step count uniform in [steps[0], steps[1]], OT or turbulence
    initial data 50/50."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        out.append(Request(i, t, int(rng.choice(edges)), int(rng.integers(steps[0], steps[1] + 1)),
                           "ot" if rng.random() < 0.5 else "turb", seed + i))
    return out


@dataclass
class _Active:
    req: Request
    handle: object
    remaining: int
    admitted: float
    nbytes: int


class Server:
    """Admission, epochs and retirement over a backend (see GpuBackend)."""

    def __init__(self, backend, budget_bytes: int, max_active: int = 64, epoch_steps: int = 10,
                 skip_ahead: int = 8, inflight: int = 2):
        self.b = backend
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.epoch_steps = epoch_steps
        self.skip_ahead = skip_ahead
        self.inflight_max = inflight

    def run(self, requests, keep_results: bool = False, progress=None):
        """Serve ``requests`` to completion; ``progress(done, total)`` is called
        after every retirement when given."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue: deque[Request] = deque()
        active: list[_Active] = []
        inflight = deque()  # (token, [_Active finishing with this epoch])
        used = 0
        done: list[Done] = []
        rejected: list[Request] = []
        t0 = self.b.now()
        peak_used = 0
        while pending or queue or active or inflight:
            now = self.b.now() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admission: FIFO with a bounded skip-ahead window
            i = 0
            while i < min(len(queue), self.skip_ahead) and len(active) < self.max_active:
                r = queue[i]
                need = self.b.workspace_bytes(r)
                if need > self.budget:
                    rejected.append(r)
                    del queue[i]
                    continue
                if used + need <= self.budget:
                    del queue[i]
                    h = self.b.open(r)
                    active.append(_Active(r, h, r.steps, self.b.now() - t0, need))
                    used += need
                    peak_used = max(peak_used, used)
                    continue
                i += 1
            # launch an epoch over every admitted box not yet finished
            runnable = [a for a in active if a.remaining > 0]
            if runnable and len(inflight) < self.inflight_max:
                n = [min(self.epoch_steps, a.remaining) for a in runnable]
                token = self.b.step([a.handle for a in runnable], n)
                finishing = []
                for a, k in zip(runnable, n):
                    a.remaining -= k
                    if a.remaining == 0:
                        finishing.append(a)
                inflight.append((token, finishing))
                continue
            # retire boxes whose last epoch has completed
            if inflight and self.b.ready(inflight[0][0]):
                _, finishing = inflight.popleft()
                tfin = self.b.now() - t0
                for a in finishing:
                    status, res = self.b.close(a.handle)
                    done.append(Done(a.req.rid, a.req.arrival, a.admitted, tfin,
                                     a.req.edge ** 3, a.req.steps, status,
                                     res if keep_results else None))
                    used -= a.nbytes
                    active.remove(a)
                if progress is not None:
                    progress(len(done), len(requests))
                continue
            # idle: wait for the GPU or the next arrival
            if inflight:
                self.b.wait(inflight[0][0], 2e-4)
            elif pending and not queue:
                self.b.sleep(max(0.0, pending[0].arrival - (self.b.now() - t0)))
            elif queue and not active:
                # nothing admitted and nothing fits: cannot happen unless budget is tiny
                rejected.extend(queue)
                queue.clear()
        makespan = self.b.now() - t0
        return Stats(done, rejected, makespan, peak_used, self.budget)


@dataclass
class Stats:
    done: list
    rejected: list
    makespan: float
    peak_bytes: int
    budget: int

    def summary(self) -> dict:
        lat = np.array([d.latency for d in self.done]) if self.done else np.zeros(1)
        cu = sum(d.cells * d.steps for d in self.done)
        return {"requests": len(self.done), "rejected": len(self.rejected),
                "failed": sum(1 for d in self.done if d.status != 0),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3),
                "makespan_s": self.makespan,
                "cell_updates_per_s": cu / self.makespan if self.makespan > 0 else 0.0,
                "peak_hbm_bytes": self.peak_bytes, "budget_bytes": self.budget}


class GpuBackend:
    """libmhd backend: one context per request on a torch workspace.  The
    initial fields (per edge and init, SERVING_VARIANTS seeded translations of
    one base field, inputs.serving_state) are generated on the host once and
    kept on the GPU, so admitting a request costs one device-to-device copy."""

    def __init__(self, precision: str = "fp32", device: str = "cuda:0", riemann: str = "hlld",
                 initial_states: dict | None = None):
        import torch

        from . import inputs as I
        from .box import MHDBox, workspace_bytes

        self.torch = torch
        self.MHDBox = MHDBox
        self._ws = workspace_bytes
        self.I = I
        self.precision = precision
        self.riemann = riemann
        self.device = device
        self.stream = torch.cuda.Stream(device)
        self._states = {} if initial_states is None else initial_states
        self._batches = {}

    def variant_state(self, edge: int, init: str, k: int, base: dict | None = None):
        key = (edge, init, k)
        if key not in self._states:
            sx, sy, sz = self.I.variant_shift(k, edge)
            if base is None:
                base = self.I.serving_base(edge, init)
            dt = self.torch.float32 if self.precision == "fp32" else self.torch.float64
            self._states[key] = {
                f: self.torch.from_numpy(np.ascontiguousarray(np.roll(v, (sz, sy, sx), axis=(0, 1, 2))))
                .to(self.device, dt) for f, v in base.items()}
        return self._states[key]

    def prepare(self, edges=EDGES, inits=("ot", "turb")):
        """Generate every variant of these edges and inits (before a replay's
        clock starts)."""
        for e in edges:
            for init in inits:
                base = self.I.serving_base(e, init)
                for k in range(self.I.SERVING_VARIANTS):
                    self.variant_state(e, init, k, base)

    def initial_state(self, r: Request):
        return self.variant_state(r.edge, r.init, self.I.request_variant(r.seed))

    def workspace_bytes(self, r: Request) -> int:
        return self._ws(r.edge, r.edge, r.edge, self.precision)

    def now(self) -> float:
        return time.perf_counter()

    def sleep(self, s: float):
        time.sleep(min(s, 0.05))

    def open(self, r: Request):
        box = self.MHDBox(r.edge, r.edge, r.edge, precision=self.precision, riemann=self.riemann,
                          device=self.device, stream=self.torch.cuda.Stream(self.device))
        box.set_state(self.initial_state(r))
        ev = self.torch.cuda.Event()
        ev.record(box.stream)
        self.stream.wait_event(ev)  # epochs run on the server stream
        return box

    def step(self, boxes, nsteps):
        import ctypes as C

        from . import _lib as L
        arr = (C.c_void_p * len(boxes))(*[b.ctx.value for b in boxes])
        n = (C.c_int * len(boxes))(*nsteps)
        L.check(boxes[0].lib.mhd_step_batch(arr, n, len(boxes), C.c_void_p(self.stream.cuda_stream)),
                "mhd_step_batch")
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def ready(self, token) -> bool:
        return token.query()

    def wait(self, token, timeout: float):
        time.sleep(timeout)

    def close(self, box):
        # the box's own stream waits for the server stream, then copies out
        box.stream.wait_stream(self.stream)
        state, t, dt, rc = box.get_state(check=False)
        box.close()
        del box.workspace
        return rc, (state, t, dt)


class MockBackend:
    """Virtual-time backend for scheduler tests: an epoch of n_i steps on boxes
    of c_i cells takes sum(c_i n_i) / rate seconds after the previous epoch."""

    def __init__(self, rate: float = 1e9, fail_rids=(), bytes_per_cell: int = 128):
        self.rate = rate
        self.t = 0.0
        self.gpu_free_at = 0.0
        self.fail = set(fail_rids)
        self.bpc = bytes_per_cell
        self.opened = []
        self.epochs = []

    def workspace_bytes(self, r):
        return r.edge ** 3 * self.bpc

    def now(self):
        return self.t

    def sleep(self, s):
        self.t += max(s, 1e-6)

    def open(self, r):
        self.opened.append(r.rid)
        return {"req": r, "steps": 0}

    def step(self, handles, nsteps):
        start = max(self.t, self.gpu_free_at)
        work = sum(h["req"].edge ** 3 * n for h, n in zip(handles, nsteps))
        self.gpu_free_at = start + work / self.rate
        for h, n in zip(handles, nsteps):
            h["steps"] += n
        self.epochs.append(([h["req"].rid for h in handles], list(nsteps)))
        return self.gpu_free_at

    def ready(self, token):
        return self.t >= token

    def wait(self, token, timeout):
        self.t = max(self.t + 1e-6, min(token, self.t + timeout * 50))

    def close(self, h):
        status = -4 if h["req"].rid in self.fail else 0
        return status, h["steps"]
