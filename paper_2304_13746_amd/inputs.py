"""Seeded synthetic initial conditions for the ideal-MHD box workloads.

This module only builds input states; it holds none of the solver's arithmetic and
imports neither the GPU library nor the CPU oracle, so both can be fed identical
arrays from it.  Every generator works in float64 with NumPy's PCG64
(``np.random.default_rng(seed)``) and returns a state dict of eight C-contiguous
arrays shaped (nz, ny, nx), x fastest:

* ``rho, mx, my, mz, en`` -- cell-centred density, momentum and total energy
  E = p/(gamma-1) + rho v^2/2 + B^2/2 (Sec. 2.1 of the paper; no 4 pi);
* ``bx, by, bz`` -- face-centred field at (i-1/2, j, k), (i, j-1/2, k),
  (i, j, k-1/2), built as the discrete curl of an edge vector potential (or
  uniform) so that its discrete divergence vanishes (constrained transport,
  Sec. 2.4).  The cell-centred field used in E is the mean of the two faces.
"""
from __future__ import annotations

import math

import numpy as np

FIELDS = ("rho", "mx", "my", "mz", "en", "bx", "by", "bz")


# ----------------------------------------------------------------- helpers

def cell_centres(n: tuple, l: tuple):
    """Cell-centre coordinates (z, y, x) broadcastable to (nz, ny, nx)."""
    nx, ny, nz = n
    lx, ly, lz = l
    x = (np.arange(nx) + 0.5) * (lx / nx)
    y = (np.arange(ny) + 0.5) * (ly / ny)
    z = (np.arange(nz) + 0.5) * (lz / nz)
    return z[:, None, None], y[None, :, None], x[None, None, :]


def face_b_from_potential(ax, ay, az, dl):
    """Face field as the discrete curl of an edge vector potential.

    ``ax[k, j, i]`` sits on the x-edge (i, j-1/2, k-1/2), ``ay`` on (i-1/2, j, k-1/2)
    and ``az`` on (i-1/2, j-1/2, k).  Stokes' theorem over each face gives a field
    whose discrete divergence is zero up to rounding.
    """
    dx, dy, dz = dl

    def dplus(a, axis):  # a[idx + 1] - a[idx] along axis, periodic
        return np.roll(a, -1, axis=axis) - a

    bx = dplus(az, 1) / dy - dplus(ay, 0) / dz
    by = dplus(ax, 0) / dz - dplus(az, 2) / dx
    bz = dplus(ay, 2) / dx - dplus(ax, 1) / dy
    return bx, by, bz


def assemble(rho, vx, vy, vz, p, bx, by, bz, gamma, shape=None):
    """Conserved state from cell primitives and face field (broadcast to ``shape``,
    default: the common shape of the inputs, which must then be 3-D)."""
    if shape is None:
        shape = np.broadcast_shapes(*(np.shape(a) for a in (rho, vx, vy, vz, p, bx, by, bz)))
    f = lambda a: np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))
    rho, vx, vy, vz, p = f(rho), f(vx), f(vy), f(vz), f(p)
    bx, by, bz = f(bx), f(by), f(bz)
    bcx = 0.5 * (bx + np.roll(bx, -1, axis=2))
    bcy = 0.5 * (by + np.roll(by, -1, axis=1))
    bcz = 0.5 * (bz + np.roll(bz, -1, axis=0))
    en = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) \
        + 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz)
    s = {"rho": rho, "mx": rho * vx, "my": rho * vy, "mz": rho * vz, "en": en,
         "bx": bx, "by": by, "bz": bz}
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in s.items()}


def to_float32_exact(s: dict) -> dict:
    """Round a state once to float32 and promote back: the common input of an
    FP32 run and of the FP64 reference it is compared with."""
    return {k: np.ascontiguousarray(v.astype(np.float32).astype(np.float64)) for k, v in s.items()}


# ------------------------------------------------------------ Orszag-Tang

def orszag_tang(n: int = 32, seed: int = 2304, gamma: float = 5.0 / 3.0, noise: float = 1e-3,
                potential: bool = False):
    """Orszag-Tang vortex (Sec. 4.2) on the periodic unit cube, extruded in z.

    rho = 25/(36 pi) (1 + noise u), u ~ U(-1, 1) seeded; p = 5/(12 pi);
    v = (-sin 2 pi y, sin 2 pi x, 0); B = B0 (-sin 2 pi y, sin 4 pi x, 0) with
    B0 = 1/sqrt(4 pi), from A_z = B0 [cos(4 pi x)/(4 pi) + cos(2 pi y)/(2 pi)].
    With ``potential`` also returns the edge potential {"ax", "ay", "az", "b0"}.
    """
    nx = ny = nz = n
    dl = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    z, y, x = cell_centres((nx, ny, nz), (1.0, 1.0, 1.0))
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    rho = 25.0 / (36.0 * math.pi) * (1.0 + noise * u)
    p = 5.0 / (12.0 * math.pi)
    vx = -np.sin(2 * math.pi * y) + 0 * x + 0 * z
    vy = np.sin(2 * math.pi * x) + 0 * y + 0 * z
    vz = 0.0
    b0 = 1.0 / math.sqrt(4 * math.pi)
    xe = np.arange(nx)[None, None, :] * dl[0]  # edge x = i dx (at i-1/2)
    ye = np.arange(ny)[None, :, None] * dl[1]
    az = b0 * (np.cos(4 * math.pi * xe) / (4 * math.pi) + np.cos(2 * math.pi * ye) / (2 * math.pi))
    az = np.broadcast_to(az, (nz, ny, nx)).copy()
    zero = np.zeros((nz, ny, nx))
    bx, by, bz = face_b_from_potential(zero, zero, az, dl)
    st = assemble(rho, vx, vy, vz, p, bx, by, bz, gamma)
    if potential:
        return st, {"ax": zero.copy(), "ay": zero.copy(), "az": az, "b0": (0.0, 0.0, 0.0)}
    return st


def orszag_tang_3d(n: int = 256, gamma: float = 5.0 / 3.0, potential: bool = False):
    """Three-dimensional Orszag-Tang performance problem (Sec. 5).

    v = (-sin 2 pi y, sin 2 pi x + cos 2 pi z, cos 2 pi x),
    B = B0 (-sin 2 pi y, sin 4 pi x, cos 2 pi x + sin 2 pi y), from the potential
    A = B0 (cos(2 pi y)/(2 pi), sin(2 pi x)/(2 pi), cos(4 pi x)/(4 pi) + cos(2 pi y)/(2 pi)).
    """
    nx = ny = nz = n
    dl = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    z, y, x = cell_centres((nx, ny, nz), (1.0, 1.0, 1.0))
    rho = 25.0 / (36.0 * math.pi)
    p = 5.0 / (12.0 * math.pi)
    tp = 2 * math.pi
    vx = -np.sin(tp * y) + 0 * x + 0 * z
    vy = np.sin(tp * x) + np.cos(tp * z) + 0 * y
    vz = np.cos(tp * x) + 0 * y + 0 * z
    b0 = 1.0 / math.sqrt(4 * math.pi)
    shape = (nz, ny, nx)
    # edge-centre coordinates: x-edges (i, j-1/2, k-1/2), y-edges (i-1/2, j, k-1/2),
    # z-edges (i-1/2, j-1/2, k)
    yf = np.arange(ny)[None, :, None] * dl[1]
    xf = np.arange(nx)[None, None, :] * dl[0]
    ax = np.broadcast_to(b0 * np.cos(tp * yf) / tp, shape).copy()
    ay = np.broadcast_to(b0 * np.sin(tp * xf) / tp, shape).copy()
    az = np.broadcast_to(b0 * (np.cos(2 * tp * xf) / (2 * tp) + np.cos(tp * yf) / tp), shape).copy()
    bx, by, bz = face_b_from_potential(ax, ay, az, dl)
    st = assemble(rho, vx, vy, vz, p, bx, by, bz, gamma)
    if potential:
        return st, {"ax": ax, "ay": ay, "az": az, "b0": (0.0, 0.0, 0.0)}
    return st


def uniform_field_potential(shape, b0):
    """Edge potential of a uniform field on a periodic box: A = 0 and the mean
    field b0 carried separately (a periodic potential has no mean curl)."""
    z = np.zeros(shape)
    return {"ax": z, "ay": z.copy(), "az": z.copy(), "b0": tuple(float(v) for v in b0)}


# ----------------------------------------------------------- turbulence

def solenoidal_field(n: tuple, seed: int, spectrum, kmin: float = 0.0, kmax: float = np.inf,
                     dtype=np.complex128):
    """Gaussian random solenoidal vector field on an (nx, ny, nz) periodic grid.

    ``spectrum(k)`` is the shell energy spectrum E(k) in units of 2 pi / L; each
    Fourier amplitude gets variance E(k) / (4 pi k^2), the k-parallel part is
    projected out and k = 0 removed.  Returns (vx, vy, vz) float64 with unit rms
    speed.
    """
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    kx = np.fft.rfftfreq(nx, d=1.0 / nx)[None, None, :]
    ky = np.fft.fftfreq(ny, d=1.0 / ny)[None, :, None]
    kz = np.fft.fftfreq(nz, d=1.0 / nz)[:, None, None]
    k2 = kx * kx + ky * ky + kz * kz
    k = np.sqrt(k2)
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where((k > 0) & (k >= kmin) & (k <= kmax),
                       np.sqrt(spectrum(np.where(k > 0, k, 1.0)) / (4 * np.pi * np.where(k > 0, k2, 1.0))),
                       0.0)
    shp = (nz, ny, nx // 2 + 1)
    comps = []
    for _ in range(3):
        re = rng.standard_normal(shp)
        im = rng.standard_normal(shp)
        comps.append(((re + 1j * im) * amp).astype(dtype))
    ksafe = np.where(k2 > 0, k2, 1.0)
    kdotv = kx * comps[0] + ky * comps[1] + kz * comps[2]
    comps[0] = comps[0] - kx * kdotv / ksafe
    comps[1] = comps[1] - ky * kdotv / ksafe
    comps[2] = comps[2] - kz * kdotv / ksafe
    del kdotv
    v = [np.fft.irfftn(c, s=(nz, ny, nx), axes=(0, 1, 2)).astype(np.float64) for c in comps]
    rms = math.sqrt(float(sum(np.mean(a * a) for a in v)))
    return tuple(a / rms for a in v)


def turbulence(n: tuple | int = 256, seed: int = 2304, kpeak: float = 4.0, mach: float = 0.5,
               rho0: float = 1.0, p0: float = 0.6, b0=(0.2, 0.0, 0.0), gamma: float = 5.0 / 3.0,
               spectrum: str = "peaked", kmin: float = 0.0, kmax: float = np.inf, l=None):
    """Uniform rho, p and B plus a seeded solenoidal velocity with rms Mach number
    ``mach`` (sound speed sqrt(gamma p / rho)).  ``spectrum`` is "peaked",
    E(k) ~ k^4 exp(-2 k^2 / kpeak^2) (maximum at k = kpeak), or "kolmogorov",
    E(k) ~ k^(-5/3) on kmin <= k <= kmax."""
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = n
    if l is None:
        h = 1.0 / max(n)
        l = (nx * h, ny * h, nz * h)
    if spectrum == "peaked":
        spec = lambda k: k ** 4 * np.exp(-2.0 * k * k / (kpeak * kpeak))
    elif spectrum == "kolmogorov":
        spec = lambda k: k ** (-5.0 / 3.0)
    else:
        raise ValueError(spectrum)
    cdt = np.complex64 if nx * ny * nz > 64 ** 3 * 64 else np.complex128
    vx, vy, vz = solenoidal_field(n, seed, spec, kmin=kmin, kmax=kmax, dtype=cdt)
    cs = math.sqrt(gamma * p0 / rho0)
    a = mach * cs
    shape = (nz, ny, nx)
    bx = np.full(shape, float(b0[0]))
    by = np.full(shape, float(b0[1]))
    bz = np.full(shape, float(b0[2]))
    s = assemble(rho0, a * vx, a * vy, a * vz, p0, bx, by, bz, gamma)
    s["_l"] = l
    return s


def sedov(n: int = 512, r_cells: float = 3.0, energy: float = 1.0, rho0: float = 1.0,
          p0: float = 1e-2, gamma: float = 5.0 / 3.0):
    """Sedov-Taylor blast (Sec. 4.1 tests): periodic unit cube, rho = 1, P = 1e-2,
    gamma = 5/3, at rest, B = 0; the cells whose centres lie within r_i =
    r_cells cell widths of the box centre get the pressure that makes the
    deposited energy sum(P dV)/(gamma - 1) equal ``energy`` (the ambient
    P = 1e-2 included)."""
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h - 0.5
    r2 = x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2
    inside = r2 < (r_cells * h) ** 2
    n_in = int(np.count_nonzero(inside))
    p_in = (gamma - 1.0) * energy / (n_in * h ** 3)
    p = np.where(inside, p_in, p0)
    z = np.zeros((n, n, n))
    return assemble(rho0, z, z, z, p, z, z, z, gamma)


def serving_base(edge: int, init: str) -> dict:
    """Base initial data of a served box of this edge: Orszag-Tang ("ot", the
    C1 form, density noise seed 2304) or turbulence ("turb", the 256^3
    benchmark's recipe at this edge, seed 2304)."""
    if init == "ot":
        return orszag_tang(edge, seed=2304)
    s = turbulence(edge, seed=2304, kpeak=4.0, mach=0.5)
    s.pop("_l")
    return s


SERVING_VARIANTS = 16


def request_variant(seed: int) -> int:
    """Which of the SERVING_VARIANTS initial fields of its edge and init a
    request's seed draws."""
    return int(np.random.default_rng(seed).integers(SERVING_VARIANTS))


def variant_shift(k: int, edge: int) -> tuple:
    """Periodic translation (sx, sy, sz), in cells, of serving variant k."""
    rng = np.random.default_rng(2304 + k)
    return tuple(int(v) for v in rng.integers(0, edge, 3))


def request_shift(seed: int, edge: int) -> tuple:
    """Periodic translation of the initial data of the request with this seed."""
    return variant_shift(request_variant(seed), edge)


def serving_state(edge: int, init: str, seed: int) -> dict:
    """Initial data of one served request: its base field translated
    periodically by the shift of the variant its seed draws (cell and face
    arrays move together, so the discrete divergence stays zero).  A server
    keeps the variants resident, so admitting a request is one copy."""
    sx, sy, sz = request_shift(seed, edge)
    return {k: np.roll(v, (sz, sy, sx), axis=(0, 1, 2)) for k, v in serving_base(edge, init).items()}


def batch_boxes(nbox: int = 64, seed: int = 2304, emin: int = 16, emax: int = 128,
                gamma: float = 5.0 / 3.0):
    """Batch of uneven periodic boxes: each edge 8 * round(e^u / 8) with
    u ~ U(ln emin, ln emax), clipped to [emin, emax]; cubic cells of size
    1 / max(n); rho = 1, p = 0.6; solenoidal velocity peaked at
    k = min(4, n_min / 8) with rms Mach ~ U(0.3, 1.0); uniform B of magnitude
    ~ U(0.05, 0.5) in an isotropic random direction.  Box b uses seed + b."""
    rng = np.random.default_rng(seed)
    boxes = []
    for b in range(nbox):
        e = np.exp(rng.uniform(math.log(emin), math.log(emax), size=3))
        dims = tuple(int(min(emax, max(emin, 8 * round(x / 8)))) for x in e)
        mach = float(rng.uniform(0.3, 1.0))
        bmag = float(rng.uniform(0.05, 0.5))
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        kp = min(4.0, min(dims) / 8.0)
        s = turbulence(dims, seed=seed + b, kpeak=kp, mach=mach, b0=tuple(bmag * d), gamma=gamma)
        boxes.append({"dims": dims, "l": s.pop("_l"), "state": s, "mach": mach, "bmag": bmag})
    return boxes


# ------------------------------------------------------------ linear waves

def mhd_primitive_jacobian(rho, u, v1, v2, bn, b1, b2, p, gamma):
    """1D ideal-MHD quasi-linear matrix A in dW/dt + A dW/dx = 0 for
    W = (rho, u, v1, v2, B1, B2, p), normal field bn constant (Sec. 2.1)."""
    A = np.zeros((7, 7))
    A[0, 0], A[0, 1] = u, rho
    A[1, 1], A[1, 4], A[1, 5], A[1, 6] = u, b1 / rho, b2 / rho, 1.0 / rho
    A[2, 2], A[2, 4] = u, -bn / rho
    A[3, 3], A[3, 5] = u, -bn / rho
    A[4, 1], A[4, 2], A[4, 4] = b1, -bn, u
    A[5, 1], A[5, 3], A[5, 5] = b2, -bn, u
    A[6, 1], A[6, 6] = gamma * p, u
    return A


LINEAR_WAVE_BOX = (3.0, 1.5, 1.5)


def linear_wave(wave: str, n: int, eps: float = 1e-6, gamma: float = 5.0 / 3.0):
    """Small-amplitude MHD eigenmode on the inclined periodic box of Sec. 4.2:
    (Lx, Ly, Lz) = (3, 1.5, 1.5), 2n x n x n cells, rho = 1, p = 3/5, B1 = 1,
    B2 = 3/2 in the rotated frame, v1 = 1 for the entropy wave and 0 otherwise.
    The wave vector is the shortest one the periodic box admits along the box
    diagonal, k = 2 pi (1/3, 2/3, 2/3), |k| = 2 pi; x1 = k/|k|.  The right-going
    eigenvector comes from the primitive Jacobian; velocity, density and pressure
    are perturbed at cell centres and B through an edge vector potential.
    Returns (state, info) with info['speed'] the wave speed and info['delta']
    the normalised eigenvector."""
    lx, ly, lz = LINEAR_WAVE_BOX
    nx, ny, nz = 2 * n, n, n
    dl = (lx / nx, ly / ny, lz / nz)
    kvec = 2 * math.pi * np.array([1.0 / lx, 1.0 / ly, 1.0 / lz])
    kmag = float(np.linalg.norm(kvec))
    x1 = kvec / kmag
    x2 = np.array([-x1[1], x1[0], 0.0])
    x2 /= np.linalg.norm(x2)
    x3 = np.cross(x1, x2)
    rho0, p0, bn, b1, b2 = 1.0, 0.6, 1.0, 1.5, 0.0
    u0 = 1.0 if wave == "entropy" else 0.0
    A = mhd_primitive_jacobian(rho0, u0, 0.0, 0.0, bn, b1, b2, p0, gamma)
    lam, R = np.linalg.eig(A)
    lam = lam.real
    R = R.real
    order = np.argsort(lam)
    lam, R = lam[order], R[:, order]
    # sorted: u-cf, u-ca, u-cs, u, u+cs, u+ca, u+cf
    idx = {"fast": 6, "alfven": 5, "slow": 4, "entropy": 3}[wave]
    vec = R[:, idx].copy()
    vec[np.abs(vec) < 1e-14] = 0.0
    vec /= np.linalg.norm(vec)
    if vec[np.argmax(np.abs(vec))] < 0:
        vec = -vec
    speed = float(lam[idx])
    drho, du, dv1, dv2, db1, db2, dp = vec
    z, y, x = cell_centres((nx, ny, nz), (lx, ly, lz))
    phase = kvec[0] * x + kvec[1] * y + kvec[2] * z
    c = np.cos(phase)
    rho = rho0 + eps * drho * c
    u = u0 + eps * du * c
    v1 = eps * dv1 * c
    v2 = eps * dv2 * c
    p = p0 + eps * dp * c
    vel = [u * x1[a] + v1 * x2[a] + v2 * x3[a] for a in range(3)]
    # B = bn x1 + b1 x2 + eps (db1 x2 + db2 x3) cos(k.x): uniform part as a face
    # constant, wave part from A = -eps sin(k.x) (k x b_hat) / |k|^2
    bhat = db1 * x2 + db2 * x3
    kxb = np.cross(kvec, bhat) / kmag ** 2
    ii = np.arange(nx)[None, None, :]
    jj = np.arange(ny)[None, :, None]
    kk = np.arange(nz)[:, None, None]
    shape = (nz, ny, nx)

    def edge_phase(ox, oy, oz):
        return kvec[0] * (ii + ox) * dl[0] + kvec[1] * (jj + oy) * dl[1] + kvec[2] * (kk + oz) * dl[2]

    ax = np.broadcast_to(-eps * np.sin(edge_phase(0.5, 0.0, 0.0)) * kxb[0], shape)
    ay = np.broadcast_to(-eps * np.sin(edge_phase(0.0, 0.5, 0.0)) * kxb[1], shape)
    az = np.broadcast_to(-eps * np.sin(edge_phase(0.0, 0.0, 0.5)) * kxb[2], shape)
    dbx, dby, dbz = face_b_from_potential(ax, ay, az, dl)
    bbg = bn * x1 + b1 * x2
    s = assemble(rho, vel[0], vel[1], vel[2], p, bbg[0] + dbx, bbg[1] + dby, bbg[2] + dbz, gamma)
    info = {"wave": wave, "speed": speed, "delta": vec, "kmag": kmag, "dims": (nx, ny, nz),
            "l": (lx, ly, lz), "eps": eps, "u0": u0, "frame": (x1, x2, x3),
            "b0": (bn, b1, b2)}
    return s, info


# ------------------------------------------------------------ shock tubes

def shock_tube_1d(n: int, left: dict, right: dict, gamma: float, axis: int = 0, l: float = 1.0):
    """Periodic double shock tube along one axis: the left state on the middle
    half of the box, the right state outside it (two mirror-image interfaces at
    l/4 and 3l/4).  States are dicts with rho, v (3), p, B (3); the normal field
    must agree on both sides."""
    shape = [1, 1, 1]
    shape[2 - axis] = n
    shape = tuple(shape)
    xc = (np.arange(n) + 0.5) * (l / n)
    inside = (xc > 0.25 * l) & (xc < 0.75 * l)

    def field(key, comp=None):
        a = np.where(inside, left[key] if comp is None else left[key][comp],
                     right[key] if comp is None else right[key][comp])
        return a.reshape(shape)

    rho, p = field("rho"), field("p")
    v = [field("v", c) for c in range(3)]
    b = [field("B", c) for c in range(3)]
    s = assemble(rho, v[0], v[1], v[2], p, b[0], b[1], b[2], gamma)
    return s
