"""FP64 CPU oracle of the ideal-MHD cell update (TEST INFRASTRUCTURE ONLY).

This package wraps ``mhd_oracle.c``, a plain, slow, step-by-step C implementation
of the Godunov finite-volume MHD cycle of Lesur et al. (arXiv:2304.13746,
Sec. 2.2-2.7).  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the GPU library never does, and
the two share no code.

``fp32_check`` (same package) compares a lower-precision stage result with the
oracle's stage, allowing only the other valid choices at E^c upwind ties.

States are dicts of eight float64 arrays shaped (nz, ny, nx): the cell-centred
conserved variables ``rho, mx, my, mz, en`` and the face-centred field ``bx`` (at
i-1/2), ``by`` (at j-1/2), ``bz`` (at k-1/2).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mhd_oracle.c")
LIB = os.path.join(HERE, "libmhd_oracle.so")
FIELDS = ("rho", "mx", "my", "mz", "en", "bx", "by", "bz")

HLLD, HLL, HLLC = 0, 1, 2
RK2, EULER, RK3 = 0, 1, 2
EMF_EC, EMF_E0, EMF_ARITH, EMF_UCT_HLL, EMF_UCT_HLLD = 0, 1, 2, 3, 4
PLM, LIMO3, PPM = 0, 1, 2
OK, ERR_INVALID_ARG, ERR_NOMEM, ERR_NONPHYSICAL = 0, -1, -2, -4

# -ffp-contract=off: no fused multiply-add, every expression rounds as written.
CFLAGS = ["-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
          "-std=c11", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libmhd_oracle.so``."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("gamma", C.c_double), ("cfl", C.c_double),
                ("riemann", C.c_int), ("integrator", C.c_int), ("emf", C.c_int),
                ("recon", C.c_int)]


class _State(C.Structure):
    _fields_ = [(f, C.POINTER(C.c_double)) for f in FIELDS]


class _Vpot(C.Structure):
    _fields_ = [("ax", C.POINTER(C.c_double)), ("ay", C.POINTER(C.c_double)),
                ("az", C.POINTER(C.c_double)), ("b0", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("MHD_ORACLE_LIB")  # alternative build (e.g. a planted mistake)
        if not path:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            path = LIB
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_max_invdt.argtypes = [C.POINTER(_Params), C.POINTER(_State), dp]
        L.orc_step.argtypes = [C.POINTER(_Params), C.POINTER(_State), dp, dp, C.c_int, C.c_double]
        L.orc_diagnostics.argtypes = [C.POINTER(_Params), C.POINTER(_State), dp]
        L.orc_mass_flux.argtypes = [C.POINTER(_Params), C.POINTER(_State), dp, dp, dp]
        L.orc_ec_tie_spread.argtypes = [C.POINTER(_Params), C.POINTER(_State), C.c_double, dp, dp,
                                        dp]
        L.orc_ec_ties.argtypes = [C.POINTER(_Params), C.POINTER(_State), C.c_double, C.c_long,
                                  C.POINTER(C.c_long), C.POINTER(C.c_int), dp, dp, dp]
        L.orc_ec_ties.restype = C.c_long
        L.orc_step_vp.argtypes = [C.POINTER(_Params), C.POINTER(_State), C.POINTER(_Vpot), dp, dp,
                                  C.c_int, C.c_double]
        L.orc_vanleer.argtypes = [C.c_double, C.c_double]
        L.orc_vanleer.restype = C.c_double
        L.orc_limo3_phi.argtypes = [C.c_double]
        L.orc_limo3_phi.restype = C.c_double
        L.orc_recon.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_ppm_faces.argtypes = [dp, dp, dp]
        for fn in (L.orc_fast_speed, L.orc_slow_speed):
            fn.argtypes = [C.c_double] * 6
            fn.restype = C.c_double
        L.orc_riemann.argtypes = [C.c_int, C.c_double, C.c_int, dp, dp, dp, dp, dp]
        L.orc_uct_hlld_coef.argtypes = [C.c_double, C.c_int, dp, dp, dp, dp]
        L.orc_uct_hlld_coef.restype = None
        L.orc_phys_flux.argtypes = [C.c_double, dp, C.c_double, dp, dp]
        L.orc_corner_emf.argtypes = [C.c_double] * 12
        L.orc_corner_emf.restype = C.c_double
        L.orc_corner_emf_scheme.argtypes = [C.c_int] + [C.c_double] * 12
        L.orc_corner_emf_scheme.restype = C.c_double
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_set_ppm_flip.argtypes = [C.c_double, C.c_long]
        L.orc_set_ppm_flip.restype = None
        L.orc_ppm_flips.restype = C.c_long
        L.orc_ppm_sites.argtypes = [C.POINTER(C.c_long), C.c_long]
        L.orc_ppm_sites.restype = C.c_long
        lp = C.POINTER(C.c_long)
        L.orc_set_ppm_pick.argtypes = [lp, lp, C.c_long, C.c_long]
        _lib = L
    return _lib


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    gamma: float = 5.0 / 3.0
    cfl: float = 0.3
    riemann: int = HLLD
    integrator: int = RK2
    emf: int = EMF_EC
    recon: int = PLM

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz, self.gamma,
                       self.cfl, self.riemann, self.integrator, self.emf, self.recon)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _cstate(p: Params, s: dict) -> _State:
    shape = (p.nz, p.ny, p.nx)
    for f in FIELDS:
        a = s[f]
        if a.dtype != np.float64 or a.shape != shape or not a.flags.c_contiguous:
            raise ValueError(f"field {f}: need C-contiguous float64 {shape}, got {a.dtype} {a.shape}")
    return _State(*[_dptr(s[f]) for f in FIELDS])


def copy_state(s: dict) -> dict:
    return {f: np.array(s[f], dtype=np.float64, order="C", copy=True) for f in FIELDS}


def max_invdt(p: Params, s: dict) -> float:
    out = C.c_double(0.0)
    rc = lib().orc_max_invdt(C.byref(p.c()), C.byref(_cstate(p, s)), C.byref(out))
    if rc not in (OK,):
        raise RuntimeError(f"orc_max_invdt failed: {rc}")
    return out.value


def step_vp(p: Params, s: dict, a: dict, t: float, dt_next: float, nsteps: int,
            t_stop: float = 0.0, check: bool = True):
    """orc_step with the field carried by the edge potential a = {"ax", "ay",
    "az", "b0"}: advances s and a in place (s's face field becomes b0 + curl A)."""
    for k in ("ax", "ay", "az"):
        assert a[k].dtype == np.float64 and a[k].flags.c_contiguous and a[k].shape == s["rho"].shape
    v = _Vpot(_dptr(a["ax"]), _dptr(a["ay"]), _dptr(a["az"]), (C.c_double * 3)(*a["b0"]))
    tt = C.c_double(t)
    dd = C.c_double(dt_next)
    rc = lib().orc_step_vp(C.byref(p.c()), C.byref(_cstate(p, s)), C.byref(v), C.byref(tt),
                           C.byref(dd), int(nsteps), float(t_stop))
    if check and rc != OK:
        raise RuntimeError(f"orc_step_vp failed: {rc}")
    return tt.value, dd.value, rc


def mass_flux(p: Params, s: dict):
    """Riemann mass flux on every (x, y, z) face of the state, three [nz][ny][nx]
    arrays (index c = face at the lower side of cell c)."""
    out = [np.zeros((p.nz, p.ny, p.nx)) for _ in range(3)]
    rc = lib().orc_mass_flux(C.byref(p.c()), C.byref(_cstate(p, s)), *[_dptr(a) for a in out])
    if rc != OK:
        raise RuntimeError(f"orc_mass_flux failed: {rc}")
    return out


def ec_tie_spread(p: Params, s: dict, band: float):
    """Per edge (sx at (i, j-1/2, k-1/2), sy at (i-1/2, j, k-1/2), sz at
    (i-1/2, j-1/2, k)): how far the E^c corner EMF of state s can move when the
    upwind switches whose |mass flux| <= band take another side (band < 0:
    |band| times the largest |mass flux| of s)."""
    out = [np.zeros((p.nz, p.ny, p.nx)) for _ in range(3)]
    rc = lib().orc_ec_tie_spread(C.byref(p.c()), C.byref(_cstate(p, s)), float(band),
                                 *[_dptr(a) for a in out])
    if rc != OK:
        raise RuntimeError(f"orc_ec_tie_spread failed: {rc}")
    return out


def ec_ties(p: Params, s: dict, band: float):
    """The E^c upwind switches of state s whose |mass flux| <= band (band < 0:
    relative to the largest |mass flux|), as arrays: edge (e n + c; e 0 E_x, 1
    E_y, 2 E_z; c the flat cell index), slot (0..3: dq1, dq3, dp1, dp3, entering
    the corner EMF as -dq1, +dq3, -dp1, +dp3 times 1/4), flux, l (taken for a
    positive flux), r (negative flux); a zero flux takes (l + r) / 2."""
    L = lib()
    ps, cs = p.c(), _cstate(p, s)
    args = (C.byref(ps), C.byref(cs), float(band))
    n = L.orc_ec_ties(*args, 0, None, None, None, None, None)
    if n < 0:
        raise RuntimeError(f"orc_ec_ties failed: {n}")
    edge = np.zeros(max(n, 1), np.int64)
    slot = np.zeros(max(n, 1), np.int32)
    flux, l, r = (np.zeros(max(n, 1)) for _ in range(3))
    m = L.orc_ec_ties(*args, n, edge.ctypes.data_as(C.POINTER(C.c_long)),
                      slot.ctypes.data_as(C.POINTER(C.c_int)), _dptr(flux), _dptr(l), _dptr(r))
    if m != n:
        raise RuntimeError(f"orc_ec_ties: {m} != {n}")
    return edge[:n], slot[:n], flux[:n], l[:n], r[:n]


def step(p: Params, s: dict, t: float, dt_next: float, nsteps: int, t_stop: float = 0.0,
         check: bool = True):
    """Advance ``s`` in place by ``nsteps`` cycles; returns (t, dt_next, rc)."""
    tt = C.c_double(t)
    dd = C.c_double(dt_next)
    rc = lib().orc_step(C.byref(p.c()), C.byref(_cstate(p, s)), C.byref(tt), C.byref(dd),
                        int(nsteps), float(t_stop))
    if check and rc != OK:
        raise RuntimeError(f"orc_step failed: {rc}")
    return tt.value, dd.value, rc


def diagnostics(p: Params, s: dict) -> dict:
    out = np.zeros(10)
    rc = lib().orc_diagnostics(C.byref(p.c()), C.byref(_cstate(p, s)), _dptr(out))
    if rc != OK:
        raise RuntimeError(f"orc_diagnostics failed: {rc}")
    return {"mass": out[0], "mom": out[1:4].copy(), "energy": out[4], "bflux": out[5:8].copy(),
            "divb_max": out[8], "divb_rms": out[9]}


def vanleer(dm: float, dp: float) -> float:
    return lib().orc_vanleer(dm, dp)


def limo3_phi(theta: float) -> float:
    return lib().orc_limo3_phi(theta)


def recon(kind: int, q0: float, q1: float, q2: float):
    """(lower, upper) face values of cell q1 between q0 and q2."""
    lo, hi = C.c_double(), C.c_double()
    lib().orc_recon(kind, q0, q1, q2, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def ppm_faces(a) -> tuple:
    """PPM (lower, upper) face values of cell a[2] from the five cells a[0..4]."""
    arr = np.ascontiguousarray(a, dtype=np.float64)
    assert arr.shape == (5,)
    lo, hi = C.c_double(), C.c_double()
    lib().orc_ppm_faces(_dptr(arr), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def uct_hlld_coef(gamma: float, wl: np.ndarray, wr: np.ndarray, bn: np.ndarray):
    """UCT-HLLD coefficients (aL, aR, dL, dR) of n faces, shape (n, 4)."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    bn = np.ascontiguousarray(bn, dtype=np.float64)
    n = bn.shape[0]
    assert wl.shape == (n, 7) and wr.shape == (n, 7)
    out = np.zeros((n, 4))
    lib().orc_uct_hlld_coef(gamma, n, _dptr(wl), _dptr(wr), _dptr(bn), _dptr(out))
    return out


def fast_speed(gamma, rho, p, bn, bt1, bt2) -> float:
    return lib().orc_fast_speed(gamma, rho, p, bn, bt1, bt2)


def slow_speed(gamma, rho, p, bn, bt1, bt2) -> float:
    return lib().orc_slow_speed(gamma, rho, p, bn, bt1, bt2)


def riemann(solver: int, gamma: float, wl: np.ndarray, wr: np.ndarray, bn: np.ndarray):
    """Face-frame Riemann fluxes for n faces: wl, wr (n, 7), bn (n,)."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    bn = np.ascontiguousarray(bn, dtype=np.float64)
    n = bn.shape[0]
    assert wl.shape == (n, 7) and wr.shape == (n, 7)
    flux = np.zeros((n, 7))
    cmax = np.zeros(n)
    lib().orc_riemann(solver, gamma, n, _dptr(wl), _dptr(wr), _dptr(bn), _dptr(flux), _dptr(cmax))
    return flux, cmax


def phys_flux(gamma: float, w, bn: float):
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.zeros(7)
    f = np.zeros(7)
    lib().orc_phys_flux(gamma, _dptr(w), bn, _dptr(u), _dptr(f))
    return u, f


def corner_emf(a1, a2, b1, b2, c00, c10, c01, c11, sq1, sq3, sp1, sp3) -> float:
    return lib().orc_corner_emf(a1, a2, b1, b2, c00, c10, c01, c11, sq1, sq3, sp1, sp3)


def corner_emf_scheme(scheme, a1, a2, b1, b2, c00, c10, c01, c11, sq1, sq3, sp1, sp3) -> float:
    return lib().orc_corner_emf_scheme(scheme, a1, a2, b1, b2, c00, c10, c01, c11, sq1, sq3,
                                       sp1, sp3)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the following oracle calls (n > 0)."""
    lib().orc_set_num_threads(int(n))


def set_ppm_flip(band: float, target: int = -1) -> None:
    """Test hook for lower-precision comparisons (Sec. 2.3, PPM): the PPM
    decisions whose outcome jumps (interface value outside its cells, extremum,
    vanishing D2) and whose test lies within ``band`` (relative to the stencil's
    largest |a|) of the threshold are counted in the order met and taken the
    other way: every one (target < 0) or only the target-th.  While band > 0
    the oracle runs on one thread, so the order is deterministic; band 0
    restores the method as written and the thread count.  Resets the count of
    ppm_flips()."""
    lib().orc_set_ppm_flip(float(band), int(target))


def ppm_flips() -> int:
    """Near PPM decisions met since the last set_ppm_flip."""
    return int(lib().orc_ppm_flips())


def ppm_sites() -> np.ndarray:
    """Site of each near decision met: d n + c for the face of direction d
    below cell c (n cells, flat [nz][ny][nx] index), 3 n + c for the edges of
    cell c formed by the edge solve."""
    n = ppm_flips()
    out = np.zeros(max(n, 1), dtype=np.int64)
    m = lib().orc_ppm_sites(out.ctypes.data_as(C.POINTER(C.c_long)), n)
    return out[:m]


def set_ppm_pick(sites, ordinals, nsite: int) -> None:
    """With a band set (set_ppm_flip): take the other way, at each of ``sites``,
    only its ``ordinals``-th near decision (counted among those met there; one
    per site); sites below ``nsite``."""
    s = np.ascontiguousarray(sites, dtype=np.int64)
    o = np.ascontiguousarray(ordinals, dtype=np.int64)
    lp = C.POINTER(C.c_long)
    rc = lib().orc_set_ppm_pick(s.ctypes.data_as(lp), o.ctypes.data_as(lp), len(s), int(nsite))
    if rc != 0:
        raise ValueError(f"orc_set_ppm_pick: {rc}")
