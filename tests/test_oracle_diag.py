"""Pins of the oracle's diagnostics (conserved totals and div B; the paper keeps
div B at round-off by constrained transport, Sec. 2.4, and reports it for the
Orszag-Tang run, Sec. 4.2) against closed forms, not against the oracle itself.

The totals are compensated (Neumaier) sums of each field times the cell volume;
div B of a cell is the sum over the three directions of the face-field
difference divided by the cell width.  Each test below fixes the answer from
arithmetic alone: exactly representable sums, a correctly rounded sum
(math.fsum), and face fields whose discrete divergence is known in closed form.
"""
import math

import numpy as np
import pytest

import oracle as O

SLOTS = ("rho", "mx", "my", "mz", "en", "bx", "by", "bz")


def const_state(shape, vals):
    return {f: np.full(shape, float(v)) for f, v in zip(SLOTS, vals)}


def flat(d):
    return [d["mass"], *d["mom"], d["energy"], *d["bflux"]]


def test_uniform_totals_exact_and_in_their_slots():
    """A uniform field q over a box of volume V totals q*V exactly when the cell
    count is a power of two (n*q and dV are then exact); each field lands in its
    own slot, so swapped outputs fail.  A plain running sum of 0.3 over 2^12
    cells is not exact, so this also pins the compensation."""
    nx, ny, nz = 16, 8, 32
    lx, ly, lz = 2.0, 0.5, 4.0
    vals = (0.3, -1.7, 0.1, 2.9, 7.3, 0.7, -0.45, 1.1)
    s = const_state((nz, ny, nx), vals)
    d = O.diagnostics(O.Params(nx, ny, nz, lx, ly, lz), s)
    vol = lx * ly * lz
    for got, v in zip(flat(d), vals):
        assert got == v * vol
    # div B of a uniform field is exactly zero
    assert d["divb_max"] == 0.0 and d["divb_rms"] == 0.0
    # the naive sum really is inexact for this input (the pin has teeth)
    naive = 0.0
    for _ in range(nx * ny * nz):
        naive += 0.3
    assert naive != 0.3 * nx * ny * nz


def test_cancellation_sum_is_exact():
    """Values 1e16, 1, -1e16 repeated (x fastest, the summation order): a plain
    running sum loses every 1; the compensated sum keeps them all."""
    n = 24  # 24^3 cells, a multiple of 3
    seq = np.tile([1e16, 1.0, -1e16], n ** 3 // 3).reshape(n, n, n)
    s = const_state((n, n, n), (1.0,) * 8)
    s["mx"] = seq.copy()
    d = O.diagnostics(O.Params(n, n, n), s)
    want = (n ** 3 // 3) * 1.0 / n ** 3  # the exact total times dV = 1/n^3
    assert d["mom"][0] == want
    naive = 0.0
    for v in seq.ravel()[:300]:
        naive += v
    assert naive != 100.0
    # the small term first: the compensation must take the branch where the
    # new term is the larger one
    s["my"] = np.tile([1.0, 1e16, -1e16], n ** 3 // 3).reshape(n, n, n)
    d = O.diagnostics(O.Params(n, n, n), s)
    assert d["mom"][1] == want


def test_random_totals_match_correctly_rounded_sum():
    """Random fields: each total is within a few ulps of the correctly rounded sum
    (math.fsum) times dV; a wrong cell volume, a dropped cell or a swapped field
    is far outside that."""
    rng = np.random.default_rng(7)
    nx, ny, nz = 12, 10, 14
    lx, ly, lz = 1.3, 0.7, 2.1
    s = {f: rng.uniform(-1.0, 3.0, (nz, ny, nx)) for f in SLOTS}
    d = O.diagnostics(O.Params(nx, ny, nz, lx, ly, lz), s)
    dv = (lx / nx) * (ly / ny) * (lz / nz)
    for got, f in zip(flat(d), SLOTS):
        want = math.fsum(s[f].ravel()) * dv
        assert abs(got - want) <= 4 * np.spacing(abs(want)), (f, got, want)


def test_planted_face_divergence_max_and_rms():
    """One x-face carries +a, one y-face +b, one z-face +c, everything else 0, on
    a box with three different cell widths.  The face i-1/2 is the lower face
    of cell i and the upper face of cell i-1, so the planted x-face gives
    div = -a/dx in cell i and +a/dx in cell i-1 (likewise in y and z).  With the
    three faces in separate cells: max = max(|a|/dx, |b|/dy, |c|/dz) and
    rms = sqrt(2 (a^2/dx^2 + b^2/dy^2 + c^2/dz^2) / ncell)."""
    nx, ny, nz = 8, 12, 10
    lx, ly, lz = 1.0, 3.0, 0.5
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    s = const_state((nz, ny, nx), (1.0, 0, 0, 0, 1.0, 0, 0, 0))
    a, b, c = 0.3, -0.8, 0.05
    s["bx"][2, 3, 4] = a   # cells (i=4) and (i=3) of row (j=3, k=2)
    s["by"][7, 6, 1] = b   # cells (j=6) and (j=5) at (i=1, k=7)
    s["bz"][5, 9, 6] = c   # cells (k=5) and (k=4) at (i=6, j=9)
    d = O.diagnostics(O.Params(nx, ny, nz, lx, ly, lz), s)
    want_max = max(abs(a) / dx, abs(b) / dy, abs(c) / dz)
    want_rms = math.sqrt(2 * ((a / dx) ** 2 + (b / dy) ** 2 + (c / dz) ** 2) / (nx * ny * nz))
    assert d["divb_max"] == pytest.approx(want_max, rel=1e-15)
    assert d["divb_rms"] == pytest.approx(want_rms, rel=1e-14)
    # the planted field carries its face flux into the totals as well
    assert d["bflux"][0] == pytest.approx(a * dx * dy * dz, rel=1e-15)
    assert d["bflux"][1] == pytest.approx(b * dx * dy * dz, rel=1e-15)
    assert d["bflux"][2] == pytest.approx(c * dx * dy * dz, rel=1e-15)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sinusoidal_face_field_divergence_closed_form(axis):
    """B_d = sin(2 pi x_d) on the d-faces (x_d = i dl at face i-1/2): the discrete
    divergence in cell i is [sin(2 pi (i+1) h) - sin(2 pi i h)]/h
    = (2 sin(pi h)/h) cos(2 pi (i+1/2) h), h = 1/n.  Over the n cell centres the
    largest |cos| is cos(pi h) and the mean of cos^2 is 1/2, so
    max = sin(2 pi h)/h and rms = sqrt(2) sin(pi h)/h."""
    dims = [16, 20, 24]
    n = dims[axis]
    h = 1.0 / n
    nx, ny, nz = dims
    s = const_state((nz, ny, nx), (1.0, 0, 0, 0, 1.0, 0, 0, 0))
    face = np.sin(2 * np.pi * np.arange(n) * h)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    s[("bx", "by", "bz")[axis]] = np.broadcast_to(face.reshape(shape), (nz, ny, nx)).copy()
    d = O.diagnostics(O.Params(nx, ny, nz), s)
    assert d["divb_max"] == pytest.approx(math.sin(2 * math.pi * h) / h, rel=1e-13)
    assert d["divb_rms"] == pytest.approx(math.sqrt(2.0) * math.sin(math.pi * h) / h, rel=1e-13)


def test_curl_of_edge_potential_is_divergence_free():
    """A face field built as the discrete curl of a random edge potential has a
    discrete divergence of zero up to rounding (Stokes' theorem on each cell,
    the property constrained transport keeps, Sec. 2.4)."""
    rng = np.random.default_rng(11)
    n = 16
    ax, ay, az = (rng.normal(size=(n, n, n)) for _ in range(3))
    h = 1.0 / n

    def dd(a, axis):  # forward difference along array axis (z=0, y=1, x=2)
        return (np.roll(a, -1, axis=axis) - a) / h

    s = const_state((n, n, n), (1.0, 0, 0, 0, 1.0, 0, 0, 0))
    # edges: ax at (i, j-1/2, k-1/2), ay at (i-1/2, j, k-1/2), az at (i-1/2, j-1/2, k)
    s["bx"] = dd(az, 1) - dd(ay, 0)
    s["by"] = dd(ax, 0) - dd(az, 2)
    s["bz"] = dd(ay, 2) - dd(ax, 1)
    d = O.diagnostics(O.Params(n, n, n), s)
    bscale = max(float(np.max(np.abs(s[f]))) for f in ("bx", "by", "bz")) / h
    assert d["divb_max"] <= 1e-14 * bscale
    assert 0.0 < d["divb_max"]  # rounding is there, and it is what is measured


def test_periodic_ramp_divergence_sign_and_norm():
    """B_x = a i on the x-faces (a ramp that wraps): cells 0..n-2 get div = +a/dx
    and the last cell -(n-1) a/dx, so the largest |div| is a negative value:
    max = (n-1) a/dx and rms = (a/dx) sqrt(n-1)."""
    nx, ny, nz = 10, 4, 6
    a, lx = 0.2, 2.0
    dx = lx / nx
    s = const_state((nz, ny, nx), (1.0, 0, 0, 0, 1.0, 0, 0, 0))
    s["bx"] = np.broadcast_to(a * np.arange(nx, dtype=float), (nz, ny, nx)).copy()
    d = O.diagnostics(O.Params(nx, ny, nz, lx, 1.0, 1.0), s)
    assert d["divb_max"] == pytest.approx((nx - 1) * a / dx, rel=1e-14)
    assert d["divb_rms"] == pytest.approx(a / dx * math.sqrt(nx - 1), rel=1e-14)
