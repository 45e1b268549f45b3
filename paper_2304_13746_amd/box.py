"""Python face of one MHD box context: torch supplies device memory and the
stream, libmhd.so does every step of the method (see include/mhd.h).

    box = MHDBox(32, 32, 32, precision="fp64", riemann="hlld")
    box.set_state(state)            # dict of 8 arrays (numpy or torch), [nz][ny][nx]
    box.step(10)                    # asynchronous on the current stream
    state, t, dt_next = box.get_state()
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

FIELDS = ("rho", "mx", "my", "mz", "en", "bx", "by", "bz")
PRECISION = {"fp64": L.MHD_FP64, "fp32": L.MHD_FP32}
RIEMANN = {"hlld": L.MHD_HLLD, "hll": L.MHD_HLL, "hllc": L.MHD_HLLC}
INTEGRATOR = {"rk2": L.MHD_RK2, "euler": L.MHD_EULER, "rk3": L.MHD_RK3}
EMF = {"ec": L.MHD_EMF_EC, "e0": L.MHD_EMF_E0, "arith": L.MHD_EMF_ARITH, "uct_hll": L.MHD_EMF_UCT_HLL,
       "uct_hlld": L.MHD_EMF_UCT_HLLD}
RECON = {"plm": L.MHD_PLM, "limo3": L.MHD_LIMO3, "ppm": L.MHD_PPM}
DTYPE = {"fp64": torch.float64, "fp32": torch.float32}


POTENTIAL = ("ax", "ay", "az")
CT = {"face": L.MHD_CT_FACE, "vecpot": L.MHD_CT_VECPOT}


def _view(tensors: dict) -> L.StateView:
    return L.StateView(*[tensors[f].data_ptr() if f in tensors else None
                         for f in FIELDS + POTENTIAL])


def make_params(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, gamma=5.0 / 3.0, cfl=0.3, precision="fp64",
                riemann="hlld", integrator="rk2", tile=0, zchunk=0, emf="ec",
                recon="plm", ct="face", b0=(0.0, 0.0, 0.0)) -> L.Params:
    p = L.Params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.lx, p.ly, p.lz = float(lx), float(ly), float(lz)
    p.gamma, p.cfl = float(gamma), float(cfl)
    p.precision = PRECISION[precision]
    p.riemann = RIEMANN[riemann]
    p.emf = EMF[emf]
    p.recon = RECON[recon]
    p.ct = CT[ct]
    p.b0 = (C.c_double * 3)(*[float(v) for v in b0])
    p.integrator = INTEGRATOR[integrator]
    p.tile, p.zchunk = int(tile), int(zchunk)
    return p


def workspace_bytes(nx, ny, nz, precision="fp64", tile=0, integrator="rk2", ct="face",
                    emf="ec") -> int:
    p = make_params(nx, ny, nz, precision=precision, tile=tile, integrator=integrator, ct=ct,
                    emf=emf)
    return int(L.lib().mhd_workspace_bytes(C.byref(p)))


class MHDBox:
    """One periodic box advanced by libmhd on a torch-owned workspace."""

    def __init__(self, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, gamma=5.0 / 3.0, cfl=0.3,
                 precision="fp64", riemann="hlld", integrator="rk2", device="cuda:0",
                 stream: torch.cuda.Stream | None = None, tile=0, zchunk=0, emf="ec",
                 recon="plm", ct="face", b0=(0.0, 0.0, 0.0)):
        self.lib = L.lib()
        self.device = torch.device(device)
        self.precision = precision
        self.dtype = DTYPE[precision]
        self.shape = (int(nz), int(ny), int(nx))
        # an explicit stream (default priority): torch's default stream may be a
        # per-thread stream that the HIP null stream does not order against
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.vecpot = ct == "vecpot"
        p = make_params(nx, ny, nz, lx, ly, lz, gamma, cfl, precision, riemann, integrator, tile,
                        zchunk, emf, recon, ct, b0)
        nbytes = int(self.lib.mhd_workspace_bytes(C.byref(p)))
        if nbytes == 0:
            raise L.MHDError(L.MHD_ERR_INVALID_ARG, "mhd_workspace_bytes")
        # torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        p.workspace = self.workspace.data_ptr()
        p.workspace_bytes = nbytes
        p.stream = self.stream.cuda_stream
        self.params = p
        self.ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.mhd_create(C.byref(p), C.byref(self.ctx)), "mhd_create")

    # ---- state in / out

    def _fields(self):
        return FIELDS + POTENTIAL if self.vecpot else FIELDS

    def _to_device(self, state: dict) -> dict:
        out = {}
        for f in self._fields():
            if self.vecpot and f in ("bx", "by", "bz") and f not in state:
                continue  # derived from the potential
            a = state[f]
            if isinstance(a, np.ndarray):
                a = np.ascontiguousarray(a)
                if not a.flags.writeable:  # torch wraps only writable arrays
                    a = a.copy()
                a = torch.from_numpy(a)
            a = a.to(device=self.device, dtype=self.dtype).contiguous()
            if tuple(a.shape) != self.shape:
                raise ValueError(f"field {f}: shape {tuple(a.shape)} != {self.shape}")
            out[f] = a
        return out

    def set_state(self, state: dict, t: float = 0.0, dt_next: float = 0.0):
        dev = self._to_device(state)
        # the inputs were produced on torch's current stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        for a in dev.values():
            a.record_stream(self.stream)
        with torch.cuda.device(self.device):
            v = _view(dev)
            L.check(self.lib.mhd_set_state(self.ctx, C.byref(v), float(t), float(dt_next)),
                    "mhd_set_state")
        return self

    def step(self, nsteps: int, t_stop: float = 0.0):
        L.check(self.lib.mhd_step(self.ctx, int(nsteps), float(t_stop)), "mhd_step")
        return self

    def get_state(self, check: bool = True):
        """Copy the state out (synchronises the box's stream)."""
        with torch.cuda.stream(self.stream):
            out = {f: torch.empty(self.shape, dtype=self.dtype, device=self.device)
                   for f in self._fields()}
        t = C.c_double()
        dt = C.c_double()
        v = _view(out)
        rc = self.lib.mhd_get_state(self.ctx, C.byref(v), C.byref(t), C.byref(dt))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        if check:
            L.check(rc, "mhd_get_state")
        return out, t.value, dt.value, rc

    def get_stage_output(self, stage: int = 1, numpy: bool = True) -> dict:
        """The last cycle's stage-`stage` result (mhd_get_stage_output), as FP64
        numpy arrays or, with numpy=False, as device tensors of the box's
        precision (synchronises the box's stream)."""
        with torch.cuda.stream(self.stream):
            out = {f: torch.empty(self.shape, dtype=self.dtype, device=self.device)
                   for f in self._fields()}
        v = _view(out)
        rc = self.lib.mhd_get_stage_output(self.ctx, int(stage), C.byref(v))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        L.check(rc, "mhd_get_stage_output")
        if not numpy:
            return out
        return {f: out[f].double().cpu().numpy() for f in out}

    def get_state_numpy(self, check: bool = True):
        s, t, dt, rc = self.get_state(check)
        return {f: s[f].double().cpu().numpy() for f in s}, t, dt, rc

    def diagnostics(self) -> dict:
        d = L.Diag()
        L.check(self.lib.mhd_get_diagnostics(self.ctx, C.byref(d)), "mhd_get_diagnostics")
        return {"mass": d.mass, "mom": np.array(d.mom[:]), "energy": d.energy,
                "bflux": np.array(d.bflux[:]), "divb_max": d.divb_max, "divb_rms": d.divb_rms,
                "status": d.status}

    # ---- launch shape

    def set_launch(self, tile: int = 0, zchunk: int = 0):
        """Tile (TILE_* constant, 0 = default) and z-planes per work-group
        (0 = automatic).  Synchronises the box's stream."""
        L.check(self.lib.mhd_set_launch(self.ctx, int(tile), int(zchunk)), "mhd_set_launch")
        return self

    def get_launch(self):
        t, z = C.c_int(), C.c_int()
        L.check(self.lib.mhd_get_launch(self.ctx, C.byref(t), C.byref(z)), "mhd_get_launch")
        return t.value, z.value

    def close(self):
        if self.ctx:
            self.lib.mhd_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
