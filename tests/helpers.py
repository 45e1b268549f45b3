"""Shared test helpers: oracle runners, error norms and state transforms."""
from __future__ import annotations

import json
import os

import numpy as np

import oracle as O
from paper_2304_13746_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name="paper_values.json"):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def run_to(p, s, t_stop, max_cycles=100000):
    """Advance the oracle one cycle at a time until t reaches t_stop."""
    t, dt = 0.0, 0.0
    n = 0
    while t < t_stop and n < max_cycles:
        t, dt, _ = O.step(p, s, t, dt, 1, t_stop)
        n += 1
    return t, n


def cell_b(s):
    return (0.5 * (s["bx"] + np.roll(s["bx"], -1, 2)),
            0.5 * (s["by"] + np.roll(s["by"], -1, 1)),
            0.5 * (s["bz"] + np.roll(s["bz"], -1, 0)))


def cons8(s):
    bcx, bcy, bcz = cell_b(s)
    return [s["rho"], s["mx"], s["my"], s["mz"], s["en"], bcx, bcy, bcz]


def linear_wave_modes(info, gamma=5.0 / 3.0):
    """Indices of the conserved cell variables (rho, m, E, B_c) that the eigenmode
    perturbs, from the linearised prim -> cons map in the grid frame."""
    x1, x2, x3 = info["frame"]
    drho, du, dv1, dv2, db1, db2, dp = info["delta"]
    v0 = info["u0"] * x1
    dv = du * x1 + dv1 * x2 + dv2 * x3
    db = db1 * x2 + db2 * x3
    bn, b1, b2 = info["b0"]
    b0 = bn * x1 + b1 * x2 + b2 * x3
    dm = 1.0 * dv + v0 * drho
    de = dp / (gamma - 1) + 0.5 * np.dot(v0, v0) * drho + np.dot(v0, dv) + np.dot(b0, db)
    du_ = [drho, *dm, de, *db]
    return [q for q in range(8) if abs(du_[q]) > 1e-10]


def linear_wave_error(s0, s1, eps, comps):
    """Error norm of the linear-wave test (Sec. 4.2): for each perturbed
    component n, the summed |dq^0 - dq^{t_c}| over cells divided by
    eps * Nx Ny Nz * N_components; the norm is the root of the sum of squares."""
    a, b = cons8(s0), cons8(s1)
    n = s0["rho"].size
    nc = len(comps)
    return float(np.sqrt(sum((np.sum(np.abs(a[q] - b[q])) / (eps * n * nc)) ** 2 for q in comps)))


def permute_xyz(s):
    """Cyclic relabelling x -> y -> z of a state: the new field at (x', y', z') is
    the old one at (x, y, z) = (y', z', x'), with vector components rotated."""
    T = lambda a: np.ascontiguousarray(np.transpose(a, (1, 2, 0)))
    return {"rho": T(s["rho"]), "en": T(s["en"]),
            "mx": T(s["mz"]), "my": T(s["mx"]), "mz": T(s["my"]),
            "bx": T(s["bz"]), "by": T(s["bx"]), "bz": T(s["by"])}


def rotate_pi_z(s):
    """Rotation by pi about the z axis, (x, y) -> (-x, -y): cell fields map
    i -> n-1-i, face fields i -> (n-i) mod n, and x, y vector components flip."""
    def cell(a):
        return np.ascontiguousarray(a[:, ::-1, ::-1])

    def xface(a):
        return np.ascontiguousarray(np.roll(a[:, ::-1, ::-1], 1, axis=2))

    def yface(a):
        return np.ascontiguousarray(np.roll(a[:, ::-1, ::-1], 1, axis=1))

    return {"rho": cell(s["rho"]), "en": cell(s["en"]), "mx": -cell(s["mx"]),
            "my": -cell(s["my"]), "mz": cell(s["mz"]), "bx": -xface(s["bx"]),
            "by": -yface(s["by"]), "bz": cell(s["bz"])}


def mirror_x(s):
    """Reflection x -> -x: cells i -> n-1-i, x-faces i -> (n-i) mod n; v_x, B_y
    and B_z change sign, B_x does not (a symmetry of the ideal-MHD equations)."""
    cell = lambda a: np.ascontiguousarray(a[:, :, ::-1])
    xface = lambda a: np.ascontiguousarray(np.roll(a[:, :, ::-1], 1, axis=2))
    return {"rho": cell(s["rho"]), "en": cell(s["en"]), "mx": -cell(s["mx"]),
            "my": cell(s["my"]), "mz": cell(s["mz"]), "bx": xface(s["bx"]),
            "by": -cell(s["by"]), "bz": -cell(s["bz"])}


def rel_err(a, b):
    """max |a - b| / max |b| (norm-wise relative difference of one field)."""
    den = float(np.max(np.abs(b)))
    if den == 0.0:
        return float(np.max(np.abs(a - b)))
    return float(np.max(np.abs(a - b))) / den


# One RK2 cycle of the scheme reads, per stage, two cells on each side of a cell
# (the van Leer slopes of both face states), so a periodic window of the state
# reproduces the whole-box result of one cycle except within 4 cells of its
# edges.  WINDOW_MARGIN leaves two more cells of slack.
WINDOW_MARGIN = 6


def window_index(center, size, dims):
    """Periodic index vectors (x, y, z) of a size^3 window whose interior
    starts at center - size // 2 on a box of dims = (nx, ny, nz)."""
    return [np.arange(center[d] - size // 2, center[d] - size // 2 + size) % dims[d]
            for d in range(3)]


def take_window(s, idx):
    """The window of every field of s (arrays [nz][ny][nx]) at idx = (ix, iy, iz)."""
    return {f: np.ascontiguousarray(s[f][np.ix_(idx[2], idx[1], idx[0])]) for f in s}


def inner(s, margin=WINDOW_MARGIN):
    sl = (slice(margin, -margin),) * 3
    return {f: s[f][sl] for f in s}


def oracle_window_cycle(s, idx, dims, l, dt, riemann=O.HLLD, gamma=5.0 / 3.0):
    """One oracle RK2 cycle with step dt on the periodic window idx of s;
    returns the window's interior (valid part)."""
    w = take_window(s, idx)
    n = [len(i) for i in idx]
    h = [l[d] / dims[d] for d in range(3)]
    p = O.Params(n[0], n[1], n[2], n[0] * h[0], n[1] * h[1], n[2] * h[2], gamma=gamma,
                 riemann=riemann)
    O.step(p, w, 0.0, dt, 1)
    return inner(w)
