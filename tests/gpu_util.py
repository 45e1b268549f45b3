"""GPU-test helpers: run the HIP library and the oracle on the same inputs."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from oracle.fp32_check import TIE_REL, best_options as _best_options, ec_tie_check  # noqa: F401
from oracle.fp32_check import stage as oracle_stage, switch_changes as ec_switch_changes  # noqa: F401

FIELDS = O.FIELDS


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_13746_amd import _lib
    _lib.lib()  # raises if libmhd.so is missing: the GPU path must be the one tested
    return torch


def gpu_box(dims, l=(1.0, 1.0, 1.0), precision="fp64", riemann="hlld", integrator="rk2",
            gamma=5.0 / 3.0, cfl=0.3, **kw):
    from paper_2304_13746_amd.box import MHDBox
    nx, ny, nz = dims
    return MHDBox(nx, ny, nz, *l, gamma=gamma, cfl=cfl, precision=precision, riemann=riemann,
                  integrator=integrator, **kw)


def oracle_params(dims, l=(1.0, 1.0, 1.0), riemann="hlld", integrator="rk2", gamma=5.0 / 3.0,
                  cfl=0.3, emf="ec", recon="plm"):
    nx, ny, nz = dims
    return O.Params(nx, ny, nz, *l, gamma=gamma, cfl=cfl,
                    riemann={"hlld": O.HLLD, "hll": O.HLL, "hllc": O.HLLC}[riemann],
                    integrator={"rk2": O.RK2, "euler": O.EULER, "rk3": O.RK3}[integrator],
                    emf={"ec": O.EMF_EC, "e0": O.EMF_E0, "arith": O.EMF_ARITH, "uct_hll": O.EMF_UCT_HLL,
                         "uct_hlld": O.EMF_UCT_HLLD}[emf],
                    recon={"plm": O.PLM, "limo3": O.LIMO3, "ppm": O.PPM}[recon])


def run_both(state, dims, nsteps, l=(1.0, 1.0, 1.0), riemann="hlld", precision="fp64",
             integrator="rk2", per_step=False, **kw):
    """Advance the same input on the GPU and in the oracle; returns
    (gpu_state, oracle_state, gpu_dts, oracle_dts) with the dt_next sequence."""
    box = gpu_box(dims, l, precision=precision, riemann=riemann, integrator=integrator, **kw)
    box.set_state(state, 0.0, 0.0)
    orc = O.copy_state(state)
    p = oracle_params(dims, l, riemann, integrator, emf=kw.get("emf", "ec"),
                      recon=kw.get("recon", "plm"))
    gd, od = [], []
    t, dt = 0.0, 0.0
    if per_step:
        for _ in range(nsteps):
            box.step(1)
            _, tg, dg, _ = box.get_state()
            gd.append(dg)
            t, dt, _ = O.step(p, orc, t, dt, 1)
            od.append(dt)
    else:
        box.step(nsteps)
        t, dt, _ = O.step(p, orc, t, dt, nsteps)
        od.append(dt)
    g, tg, dg, _ = box.get_state_numpy()
    if not per_step:
        gd.append(dg)
    box.close()
    return g, orc, gd, od, (tg, t)


GROUPS = (("rho",), ("mx", "my", "mz"), ("en",), ("bx", "by", "bz"))


def max_rel(g, o):
    """Largest norm-wise relative difference: for each quantity (density,
    momentum vector, energy, field vector) max|g - o| over its components
    divided by the largest |o| over those components."""
    worst = 0.0
    for grp in GROUPS:
        den = max(max(float(np.max(np.abs(o[f]))) for f in grp), 1e-300)
        num = max(float(np.max(np.abs(g[f] - o[f]))) for f in grp)
        worst = max(worst, num / den)
    return worst


def bit_equal(g, o):
    return all(np.array_equal(g[f], o[f]) for f in FIELDS)


STAGE_WEIGHTS = {"rk2": [(1.0, 0.0), (0.5, 0.5)], "euler": [(1.0, 0.0)],
                 "rk3": [(1.0, 0.0), (0.25, 0.75), (2.0 / 3.0, 1.0 / 3.0)]}


# ---- a bound on E^c tie effects (tested in test_fp32_ties.py; the stage checks
# match each departure exactly, oracle.fp32_check.ec_tie_check)
#
# Within one stage the corner EMF is a quarter of a sum of upwinded terms, so a
# switch that takes the other side moves it by at most a quarter of |L - R| of
# that switch (oracle.ec_tie_spread sums this over the switches whose mass flux
# lies within `band` of zero).  The face-field update of the stage is a
# difference of corner EMFs times dt/dl, so its possible departure from the
# oracle's value is at most the slack below.


def ec_field_slack(p, s, dt, band=None, band_rel=TIE_REL, weight=1.0):
    """Per face-field array: the largest change one stage of step dt from s can
    show when the E^c switches within `band` (default band_rel of the largest
    mass flux) take another side, times the stage weight."""
    sx, sy, sz = O.ec_tie_spread(p, s, -band_rel if band is None else band)
    tx, ty, tz = dt * p.nx / p.lx, dt * p.ny / p.ly, dt * p.nz / p.lz

    def up(a, axis):  # value at the next index along an array axis (z=0, y=1, x=2)
        return np.roll(a, -1, axis=axis)

    return {"bx": weight * (ty * (up(sz, 1) + sz) + tz * (up(sy, 0) + sy)),
            "by": weight * (tz * (up(sx, 0) + sx) + tx * (up(sz, 2) + sz)),
            "bz": weight * (tx * (up(sy, 2) + sy) + ty * (up(sx, 1) + sx))}


# ---- stage-wise FP32 validity
#
# An FP32 run cannot follow the FP64 oracle over many cycles where the method
# takes discontinuous decisions (the E^c upwind switch), so it is checked one
# stage at a time: each stage output of the GPU is compared with the oracle's
# stage applied to the GPU's own (FP32) input of that stage, with the GPU's step.
# Fluid variables must agree to `tol` (density and energy element by element,
# momentum norm-wise against the largest |m|); face fields to `tol` of the
# largest |B|, except where E^c switches whose mass flux lies within rounding of
# zero took another, equally valid choice: each such departure must be what
# some choice at the switches around it gives (ec_tie_check below).


def stage_errors(got, want, slack=None, tol=1e-5):
    """Errors of one FP32 stage output against the oracle stage (see above).
    b_excess: largest (|dB| - slack) / max|B| (must stay <= tol); b_tie_faces:
    faces whose |dB| needed the slack."""
    e = {}
    for f in ("rho", "en"):
        e[f] = float(np.max(np.abs(got[f] - want[f]) / np.abs(want[f])))
    mscale = max(max(float(np.max(np.abs(want[f]))) for f in ("mx", "my", "mz")), 1e-300)
    e["m"] = max(float(np.max(np.abs(got[f] - want[f]))) for f in ("mx", "my", "mz")) / mscale
    bscale = max(max(float(np.max(np.abs(want[f]))) for f in ("bx", "by", "bz")), 1e-300)
    excess, plain, ties = 0.0, 0.0, 0
    for f in ("bx", "by", "bz"):
        d = np.abs(got[f] - want[f])
        plain = max(plain, float(np.max(d)) / bscale)
        sl = slack[f] if slack is not None else 0.0
        excess = max(excess, float(np.max(d - sl)) / bscale)
        ties += int(np.count_nonzero(d > tol * bscale))
    e["b"] = plain
    e["b_excess"] = excess
    e["b_tie_faces"] = ties
    return e


def assert_stage_valid(e, tol=1e-5):
    for k in ("rho", "en", "m", "b_excess"):
        assert e[k] <= tol, e


def check_fp32_cycles(box, p, ncycles, integrator="rk2", tol=1e-5, weights=None):
    """Advance the FP32 box ncycles cycles one at a time; after each, check every
    stage (see above) and the step measured during it.  Returns the worst errors
    over all stages and cycles."""
    ws = weights or STAGE_WEIGHTS[integrator]
    x0, _, dt, rc = box.get_state_numpy()
    assert rc == 0
    worst = {}
    for c in range(ncycles):
        box.step(1)
        mids = [box.get_stage_output(k) for k in range(1, len(ws))]
        y, _, dt_new, rc = box.get_state_numpy()
        assert rc == 0
        ins, outs = [x0] + mids, mids + [y]
        for k, (w, w0) in enumerate(ws):
            e = check_fp32_stage(p, ins[k], dt, outs[k], w, w0, x0, tol)
            print(f"cycle {c} stage {k + 1}: {e}", flush=True)
            for key, v in e.items():
                worst[key] = max(worst.get(key, 0), v)
        # the step of the next cycle: measured on x0 during the first stage
        want_dt = p.cfl / O.max_invdt(p, x0)
        assert abs(dt_new - want_dt) <= tol * want_dt, (dt_new, want_dt)
        x0, dt = y, dt_new
    return worst


# ---- stage-wise FP32 validity for PPM (reading R21)
#
# Three PPM decisions make a face value jump when they change (an interface
# value outside the interval of its two cells, a cell at an extremum, D2 = 0),
# so where one of them sits within FP32 rounding of its threshold an FP32 stage
# can take the other, equally valid outcome and move the cells next to that face
# by far more than rounding.  The oracle's test hook (oracle.set_ppm_flip) finds
# every such near decision of a stage (its test within PPM_BAND of the threshold,
# relative to its stencil, and its two outcomes different) and takes any chosen
# ones the other way.  A stage is valid when every cell that departs from the
# oracle stage by more than `tol` is matched, in all eight fields at once and
# to `tol`, by the oracle stage with some subset of the near decisions around
# it taken the other way, and under E^c some choice at the switches near ties
# around it (ec_tie_check; the changes add: each decision moves one face's
# states, each switch one edge EMF).  Decisions and choices that move a cell by
# less than 1e-3 tol are not enumerated but added to its allowance.

PPM_BAND = 1e-6  # about 16 FP32 ulps of the stencil's largest value


def _cheb(cells, cell, shape):
    """Chebyshev distance on the periodic grid between flat cell indices."""
    nz, ny, nx = shape
    k, j, i = cells // (nx * ny), (cells // nx) % ny, cells % nx
    kb, jb, ib = cell // (nx * ny), (cell // nx) % ny, cell % nx
    dk = np.abs((k - kb + nz // 2) % nz - nz // 2)
    dj = np.abs((j - jb + ny // 2) % ny - ny // 2)
    di = np.abs((i - ib + nx // 2) % nx - nx // 2)
    return np.maximum(np.maximum(dk, dj), di)


def _best_subset(r0, V, al):
    """min over subsets S of the rows of V of max_f |r0 - sum_S V| - al."""
    return _best_options(r0, [np.vstack([np.zeros(len(r0)), v]) for v in V], al)


def ppm_flip_check(p, x, dt, got, w=1.0, w0=0.0, base=None, tol=1e-5, band=PPM_BAND, ec=False,
                   small=1e-3, maxk=22):
    """Check one FP32 PPM stage output `got` of input `x` (see above); with
    `ec`, the choices at E^c switches near ties (ec_tie_check) join the near PPM
    decisions around each departing cell.  Returns counts: cells above tol,
    near decisions, candidates, oracle runs, cells no choice explains (or with
    more than maxk decisions of consequence around them), and the largest
    remaining error."""
    want = oracle_stage(p, x, dt, w, w0, base)
    shape = got["rho"].shape
    ncell = int(np.prod(shape))
    # a decision at a face moves that face's flux: the two cells beside it, and
    # through the edge EMFs the face fields one cell further
    reach = 1 if p.riemann == O.HLLC else 2
    scale = {}
    for grp in GROUPS:
        sc = max(max(float(np.max(np.abs(want[f]))) for f in grp), 1e-300)
        for f in grp:
            scale[f] = sc
    den = {f: (np.abs(want[f]) if f in ("rho", "en") else np.full(shape, scale[f])) for f in FIELDS}
    resid = {f: (got[f] - want[f]) / den[f] for f in FIELDS}
    bad = np.zeros(shape, bool)
    for f in FIELDS:
        bad |= np.abs(resid[f]) > tol
    bcell = np.flatnonzero(bad)
    out = {"bad": int(len(bcell)), "near": 0, "candidates": 0, "runs": 0, "unexplained": 0,
           "residual": 0.0, "most_decisions": 0}
    if len(bcell) == 0:
        return out
    try:
        O.set_ppm_flip(band, 1 << 60)  # count and locate, take none the other way
        oracle_stage(p, x, dt, w, w0, base)
        sites = O.ppm_sites()
        out["near"] = int(len(sites))
        start = np.r_[0, np.flatnonzero(np.diff(sites) != 0) + 1]
        ords = np.arange(len(sites)) - np.repeat(start, np.diff(np.r_[start, len(sites)]))
        cells = sites % ncell
        near_bad = np.zeros(len(sites), bool)
        for b in bcell:
            near_bad |= _cheb(cells, b, shape) <= reach
        cand = np.flatnonzero(near_bad)
        out["candidates"] = int(len(cand))
        # one oracle run per group of candidates more than 2 reach apart: no
        # departing cell is within reach of two decisions of a group
        groups = []
        for c in cand:
            for g in groups:
                if np.all(_cheb(cells[g], cells[c], shape) > 2 * reach):
                    g.append(c)
                    break
            else:
                groups.append([c])
        out["runs"] = len(groups)
        delta = {n: [] for n in range(len(bcell))}
        at = [np.unravel_index(b, shape) for b in bcell]
        for g in groups:
            g = np.array(g)
            O.set_ppm_flip(band, 1 << 60)
            O.set_ppm_pick(sites[g], ords[g], 4 * ncell)
            alt = oracle_stage(p, x, dt, w, w0, base)
            for n, b in enumerate(bcell):
                if not np.any(_cheb(cells[g], b, shape) <= reach):
                    continue
                v = np.array([(alt[f][at[n]] - want[f][at[n]]) / den[f][at[n]] for f in FIELDS])
                if np.any(v != 0):
                    delta[n].append(v)
    finally:
        O.set_ppm_flip(0.0)
    # E^c switches near ties: per departing cell, the face-field changes of
    # their other choices
    ec_items = {n: [] for n in range(len(bcell))}
    if ec:
        changes = ec_switch_changes(p, O.ec_ties(p, x, -TIE_REL), dt, w)
        where = {int(b): n for n, b in enumerate(bcell)}
        for per_alt in changes:
            opts = {}
            for a, ch in enumerate(per_alt):
                for comp, c, v in ch:
                    if c in where:
                        opts.setdefault(where[c], np.zeros((1 + len(per_alt), len(FIELDS))))
                        opts[where[c]][1 + a, FIELDS.index(comp)] += v / scale[comp]
            for n, o in opts.items():
                ec_items[n].append(o)
    for n in range(len(bcell)):
        r0 = np.array([resid[f][at[n]] for f in FIELDS])
        al = np.zeros(len(FIELDS))
        big = [v for v in delta[n] if np.max(np.abs(v)) > small * tol]
        for v in delta[n]:
            if np.max(np.abs(v)) <= small * tol:
                al = al + np.abs(v)
        items = [np.vstack([np.zeros(len(FIELDS)), v]) for v in big]
        for o in ec_items[n]:  # E^c choices of no consequence join the allowance
            if np.max(np.abs(o)) > small * tol:
                items.append(o)
            else:
                al = al + np.max(np.abs(o), axis=0)
        out["most_decisions"] = max(out["most_decisions"], len(items))
        best = _best_options(r0, items, al) if len(big) <= maxk else np.inf
        out["residual"] = max(out["residual"], best)
        if not best <= tol:
            out["unexplained"] += 1
    return out


def check_fp32_ppm_cycles(box, p, ncycles, integrator="rk3", tol=1e-5):
    """check_fp32_cycles for PPM: every stage by ppm_flip_check (with the E^c
    switch choices under E^c).  Returns the totals over all stages."""
    ws = STAGE_WEIGHTS[integrator]
    x0, _, dt, rc = box.get_state_numpy()
    assert rc == 0
    tot = {"bad": 0, "near": 0, "candidates": 0, "runs": 0, "unexplained": 0, "residual": 0.0,
           "most_decisions": 0}
    for c in range(ncycles):
        box.step(1)
        mids = [box.get_stage_output(k) for k in range(1, len(ws))]
        y, _, dt_new, rc = box.get_state_numpy()
        assert rc == 0
        ins, outs = [x0] + mids, mids + [y]
        for k, (w, w0) in enumerate(ws):
            r = ppm_flip_check(p, ins[k], dt, outs[k], w, w0, x0, tol=tol,
                               ec=p.emf == O.EMF_EC and p.riemann != O.HLLC)
            print(f"cycle {c} stage {k + 1}: {r}", flush=True)
            assert r["unexplained"] == 0, (c, k + 1, r)
            for key, v in r.items():
                tot[key] = max(tot[key], v) if key in ("residual", "most_decisions") else tot[key] + v
        want_dt = p.cfl / O.max_invdt(p, x0)
        assert abs(dt_new - want_dt) <= tol * want_dt, (dt_new, want_dt)
        x0, dt = y, dt_new
    return tot


def check_fp32_stage(p, x, dt, got, w=1.0, w0=0.0, base=None, tol=1e-5, mask=None):
    """One FP32 stage against the oracle's stage on the same input: fluid to
    tol (stage_errors), face fields to tol up to E^c ties (ec_tie_check), on the
    cells of mask (default all).  Returns the errors; asserts validity."""
    want = oracle_stage(p, x, dt, w, w0, base)
    sel = (lambda d: {f: v[mask] for f, v in d.items()}) if mask is not None else (lambda d: d)
    e = stage_errors(sel(got), sel(want), None, tol)
    if p.emf == O.EMF_EC and p.riemann != O.HLLC:
        t = ec_tie_check(p, x, dt, got, w, w0, base, tol, want=want, mask=mask)
        e.update(t)
        e["b_excess"] = t["b_residual"]
        assert t["b_unexplained"] == 0, e
    assert_stage_valid(e, tol)
    return e
