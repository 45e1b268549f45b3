"""Checks of a lower-precision stage result against the oracle (TEST
INFRASTRUCTURE ONLY: used by the test suite and the benchmark's comparison with
the oracle; the GPU library never imports it).

E^c upwind ties (Sec. 2.4): the corner EMF is a quarter of the four face EMFs
plus four upwinded derivative terms; each term picks one of two candidates by
the sign of a face mass flux, their mean where the flux is zero.  Where that
flux lies within FP32 rounding of zero an FP32 stage may take either candidate
or the mean.  ``ec_ties`` (the oracle) lists those switches with their
candidates; the change that another choice makes to the face fields of the
stage follows from the corner-EMF formula and the discrete Stokes update alone
(linear in the EMF), so no further oracle run is needed.  A face-field
departure above ``tol`` must be matched, for the three faces of its cell at once
and to ``tol``, by some choice at the switches around it (choices that move the
cell by less than 1e-3 tol are added to its allowance instead of enumerated).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import EULER, FIELDS, copy_state, ec_ties, step

TIE_REL = 1e-5  # band of the E^c switches near ties, relative to the largest mass flux


def stage(p, x, dt, w=1.0, w0=0.0, base=None):
    """w S_dt(x) + w0 base with S_dt one stage of the oracle (an Euler cycle of
    step dt); the combination in FP64 numpy."""
    pe = dataclasses.replace(p, integrator=EULER)
    y = copy_state(x)
    step(pe, y, 0.0, dt, 1)
    if w == 1.0 and w0 == 0.0:
        return y
    return {f: w * y[f] + w0 * base[f] for f in FIELDS}


# (component, cell offset (dz, dy, dx), coefficient in units of tau_d) of the
# face fields that an edge EMF change moves, per edge kind (0 E_x, 1 E_y, 2 E_z)
# and stage step tau = dt / dl: the Stokes update of the stage operator
EDGE_STENCIL = {
    2: (("bx", (0, 0, 0), "y", 1.0), ("bx", (0, -1, 0), "y", -1.0),
        ("by", (0, 0, 0), "x", -1.0), ("by", (0, 0, -1), "x", 1.0)),
    1: (("bx", (0, 0, 0), "z", -1.0), ("bx", (-1, 0, 0), "z", 1.0),
        ("bz", (0, 0, 0), "x", 1.0), ("bz", (0, 0, -1), "x", -1.0)),
    0: (("by", (0, 0, 0), "z", 1.0), ("by", (-1, 0, 0), "z", -1.0),
        ("bz", (0, 0, 0), "y", -1.0), ("bz", (0, -1, 0), "y", 1.0)),
}


def switch_changes(p, ties, dt, weight=1.0, alternatives="both"):
    """For each listed switch, the face-field changes of the stage if it takes
    another choice: a list per switch of [(component, flat cell, change) for
    each alternative].  alternatives "both": the two choices it did not take;
    "mean": the mean of the candidates only (the E^0 value)."""
    edge, slot, flux, l, r = ties
    n = p.nx * p.ny * p.nz
    shape = (p.nz, p.ny, p.nx)
    tau = {"x": dt * p.nx / p.lx, "y": dt * p.ny / p.ly, "z": dt * p.nz / p.lz}
    mean = 0.5 * (l + r)
    chosen = np.where(flux > 0, l, np.where(flux < 0, r, mean))
    if alternatives == "mean":
        alts = [mean]
    else:
        alts = [np.where(flux > 0, r, l), np.where(flux == 0, r, mean)]
    sgn = np.where((slot == 0) | (slot == 2), -1.0, 1.0)
    kind, cell = edge // n, edge % n
    kk, jj, ii = np.unravel_index(cell, shape)
    out = []
    for q in range(len(edge)):
        per_alt = []
        for a in alts:
            de = 0.25 * sgn[q] * (a[q] - chosen[q]) * weight
            ch = []
            for comp, (dk, dj, di), ax, coef in EDGE_STENCIL[int(kind[q])]:
                c = np.ravel_multi_index(((kk[q] + dk) % p.nz, (jj[q] + dj) % p.ny,
                                          (ii[q] + di) % p.nx), shape)
                ch.append((comp, int(c), coef * tau[ax] * de))
            per_alt.append(ch)
        out.append(per_alt)
    return out


def _option_sums(items, width):
    s = np.zeros((1, width))
    for opt in items:
        s = (s[:, None, :] + opt[None, :, :]).reshape(-1, width)
    return s


def best_options(r0, items, al, limit=1 << 24):
    """min over one row of each item's option matrix (every item's first row is
    zero: no change) of max_f |r0 - sum| - al.  All combinations: the sums of
    the two halves' combinations met pairwise, in chunks; inf beyond `limit`
    combinations."""
    if np.prod([float(len(o)) for o in items]) > limit:
        return np.inf
    halves, size = ([], []), [1, 1]
    for opt in sorted(items, key=len, reverse=True):
        k = 0 if size[0] <= size[1] else 1
        halves[k].append(opt)
        size[k] *= len(opt)
    a, b = _option_sums(halves[0], len(r0)), _option_sums(halves[1], len(r0))
    t = r0 - a
    best = np.inf
    for i in range(0, len(t), 256):
        e = np.max(np.abs(t[i:i + 256, None, :] - b[None, :, :]) - al, axis=2)
        best = min(best, float(e.min()))
    return best


def ec_tie_check(p, x, dt, got, w=1.0, w0=0.0, base=None, tol=1e-5, band_rel=TIE_REL, maxk=14,
                 want=None, mask=None, small=1e-3):
    """Check the face fields of one FP32 stage output `got` of input `x` under
    E^c (see above), on the cells of `mask` (default all); returns counts of
    departing cells, switches near ties, cells no choice explains, and the
    largest remaining error (b_residual: at most tol when every cell is
    explained, else the largest departure)."""
    if want is None:
        want = stage(p, x, dt, w, w0, base)
    comps = ("bx", "by", "bz")
    sel = (lambda a: a[mask]) if mask is not None else (lambda a: a)
    bsc = max(max(float(np.max(np.abs(sel(want[f])))) for f in comps), 1e-300)
    resid = {f: (got[f] - want[f]) / bsc for f in comps}
    bad = np.zeros(got["bx"].shape, bool)
    for f in comps:
        bad |= np.abs(resid[f]) > tol
    if mask is not None:
        bad &= mask
    out = {"b_bad": int(bad.sum()), "ties": 0, "b_unexplained": 0,
           "b_residual": max(float(np.max(np.abs(sel(resid[f])))) for f in comps),
           "most_switches": 0}
    if not bad.any():
        return out
    out["b_residual"] = max(float(np.max(np.abs(sel(resid[f])[~sel(bad)]))) for f in comps) \
        if (~sel(bad)).any() else 0.0
    ties = ec_ties(p, x, -band_rel)
    out["ties"] = int(len(ties[0]))
    changes = switch_changes(p, ties, dt, w)
    # which switches move which cell
    touch = {}
    for q, per_alt in enumerate(changes):
        for comp, c, v in per_alt[0]:
            touch.setdefault(c, set()).add(q)
    flat = {f: resid[f].ravel() for f in comps}
    for c in np.flatnonzero(bad.ravel()):
        qs = sorted(touch.get(int(c), ()))
        out["most_switches"] = max(out["most_switches"], len(qs))
        r0 = np.array([flat[f][c] for f in comps])
        options, al = [], np.zeros(3)
        for q in qs:
            opt = np.zeros((1 + len(changes[q]), 3))
            for a, ch in enumerate(changes[q]):
                for comp, cc, v in ch:
                    if cc == c:
                        opt[1 + a, comps.index(comp)] += v / bsc
            if np.max(np.abs(opt)) > small * tol:
                options.append(opt)
            else:  # choices of no consequence join the allowance
                al = al + np.max(np.abs(opt), axis=0)
        best = best_options(r0, options, al) if len(options) <= maxk else np.inf
        out["b_residual"] = max(out["b_residual"], best)
        if not best <= tol:
            out["b_unexplained"] += 1
    return out
