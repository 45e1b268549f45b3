"""PPM reconstruction (Sec. 2.3; Colella & Woodward 1984 with the Colella &
Sekora 2008 extremum limiter) on the GPU against the FP64 oracle.

The stage kernel widens its LDS halo to three cells and its z-window to five
planes for PPM; these cases cross tile and z-chunk boundaries, wrap the
periodic halo more than once around a two-cell extent, and run every tile
shape.  FP64 must be bit-identical; the FP32 bounds are derived in the FP32
tests below.
"""
import pytest

import numpy as np

from gpu_util import GROUPS, bit_equal, gpu_box, max_rel, need_gpu, run_both
from paper_2304_13746_amd import _lib as L
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("integrator", ["rk2", "rk3"])
@pytest.mark.parametrize("riemann", ["hlld", "hll"])
def test_ppm_fp64_bit_exact(riemann, integrator):
    need_gpu()
    dims = (40, 24, 18)
    s = I.turbulence(dims, seed=23, kpeak=2.0, mach=1.0, b0=(0.2, 0.3, -0.1))
    l = s.pop("_l")
    print("ppm", riemann, integrator, dims, flush=True)
    g, o, gd, od, (tg, to) = run_both(s, dims, 4, l=l, riemann=riemann, integrator=integrator,
                                      per_step=True, recon="ppm", zchunk=5)
    print("max rel", max_rel(g, o))
    assert bit_equal(g, o)
    assert gd == od and tg == to


@pytest.mark.parametrize("tile", [L.TILE_16x16, L.TILE_24x8, L.TILE_18x11])
def test_ppm_fp64_every_tile(tile):
    need_gpu()
    dims = (37, 29, 11)
    s = I.turbulence(dims, seed=29, kpeak=2.0, mach=0.9, b0=(0.1, -0.2, 0.25))
    l = s.pop("_l")
    print("ppm tile", tile, dims, flush=True)
    g, o, gd, od, _ = run_both(s, dims, 3, l=l, per_step=True, recon="ppm", tile=tile, zchunk=4)
    assert bit_equal(g, o)
    assert gd == od


@pytest.mark.parametrize("emf", ["ec", "uct_hll"])
@pytest.mark.parametrize("dims", [(2, 9, 5), (7, 2, 3), (5, 6, 2), (1, 1, 33)])
def test_ppm_fp64_narrow_boxes(dims, emf):
    """Extents of one and two cells: the three-cell halo (and, with UCT-HLL, the
    six-face edge lines) wraps the box more than once, exactly as the oracle's
    periodic index does."""
    need_gpu()
    s = I.turbulence(dims, seed=31, kpeak=1.0, mach=0.7, b0=(0.3, 0.1, 0.2))
    l = s.pop("_l")
    print("ppm narrow", dims, emf, flush=True)
    g, o, gd, od, _ = run_both(s, dims, 3, l=l, per_step=True, recon="ppm", zchunk=2, emf=emf)
    assert bit_equal(g, o)
    assert gd == od


def test_ppm_sedov_hllc_fp64_bit_exact():
    """The hydrodynamic path (HLLC, B = 0) with PPM on the Sedov-Taylor blast."""
    need_gpu()
    n = 36
    s = I.sedov(n)
    print("ppm sedov hllc", n, flush=True)
    g, o, gd, od, (tg, to) = run_both(s, (n, n, n), 5, riemann="hllc", per_step=True,
                                      recon="ppm", integrator="rk3")
    assert bit_equal(g, o)
    assert gd == od and tg == to
    for f in ("bx", "by", "bz"):
        assert not g[f].any()


def _group_stats(g, o):
    """Per quantity group: max relative error, L2 relative error, and the
    fraction of cells whose error exceeds 1e-5 of the group's largest value."""
    out = {}
    for grp in GROUPS:
        scale = max(float(np.max(np.abs(o[f]))) for f in grp)
        err = np.max([np.abs(g[f] - o[f]) for f in grp], axis=0)
        l2 = np.sqrt(sum(float(np.sum((g[f] - o[f]) ** 2)) for f in grp) /
                     sum(float(np.sum(o[f] ** 2)) for f in grp))
        out[grp[0]] = (float(err.max()) / scale, float(l2), float(np.mean(err > 1e-5 * scale)))
    return out


@pytest.mark.parametrize("riemann", ["hlld", "hll"])
def test_ppm_fp32_within_tolerance(riemann):
    """FP32 PPM against the FP64 oracle on Orszag-Tang 32^3, 5 RK3 cycles.

    The PPM limiters switch branches on sign tests of differences, and a switch
    moves a face value discontinuously, so FP32 rounding that flips one moves a
    few cells by more than FP32 rounding otherwise would (an FP32 build of the
    same CPU algorithm differs from the FP64 one by 3.5e-5 at its worst cell, by
    4.6e-7 in L2, with 9e-5 of the cells above 1e-5).  The bounds: L2 relative
    2e-6, worst cell 2e-4, at most 1e-3 of the cells above 1e-5."""
    need_gpu()
    s = I.to_float32_exact(I.orszag_tang(32))
    print("ppm fp32", riemann, flush=True)
    g, o, _, _, _ = run_both(s, (32, 32, 32), 5, riemann=riemann, precision="fp32", recon="ppm",
                             integrator="rk3")
    st = _group_stats(g, o)
    print("ppm fp32 (max rel, l2 rel, fraction > 1e-5)", riemann, st)
    for name, (mx, l2, frac) in st.items():
        assert l2 <= 2e-6 and mx <= 2e-4 and frac <= 1e-3, (name, mx, l2, frac)


@pytest.mark.parametrize("emf", ["e0", "arith", "uct_hll"])
def test_ppm_fp32_other_emf_schemes(emf):
    """FP32 PPM with the corner-EMF schemes that take no upwind decision, on the
    same Orszag-Tang run: held to the same PPM bounds as with E^c."""
    need_gpu()
    s = I.to_float32_exact(I.orszag_tang(32))
    print("ppm fp32", emf, flush=True)
    g, o, _, _, _ = run_both(s, (32, 32, 32), 5, precision="fp32", recon="ppm", integrator="rk3",
                             emf=emf)
    st = _group_stats(g, o)
    print("ppm fp32 (max rel, l2 rel, fraction > 1e-5)", emf, st)
    for name, (mx, l2, frac) in st.items():
        assert l2 <= 2e-6 and mx <= 2e-4 and frac <= 1e-3, (name, mx, l2, frac)


def test_ppm_sedov_hllc_fp32():
    """FP32 PPM on the Sedov-Taylor blast.  One Euler cycle agrees with the
    oracle to 1e-5; over several RK3 cycles the strong shock makes the limiter
    branches sensitive to rounding (an FP32 build of the CPU algorithm already
    departs from the FP64 one by 12% at single cells after 5 cycles), so the
    longer run is checked by what rounding cannot change: finite, positive
    density and pressure, mass and energy conserved to FP32 rounding, and the
    field exactly zero."""
    need_gpu()
    n = 32
    s = I.to_float32_exact(I.sedov(n))
    print("ppm sedov hllc fp32 euler", flush=True)
    g, o, gd, od, _ = run_both(s, (n, n, n), 1, riemann="hllc", precision="fp32", recon="ppm",
                               integrator="euler")
    assert max_rel(g, o) <= 1e-5
    print("ppm sedov hllc fp32 rk3", flush=True)
    box = gpu_box((n, n, n), precision="fp32", riemann="hllc", recon="ppm", integrator="rk3")
    box.set_state(s)
    box.step(5)
    g, _, _, rc = box.get_state_numpy()
    box.close()
    assert rc == 0
    ke = 0.5 * (g["mx"] ** 2 + g["my"] ** 2 + g["mz"] ** 2) / g["rho"]
    p = (5.0 / 3.0 - 1.0) * (g["en"] - ke)
    assert np.isfinite(p).all() and g["rho"].min() > 0 and p.min() > 0
    for f in ("rho", "en"):
        tot0, tot = float(np.sum(s[f])), float(np.sum(g[f]))
        assert abs(tot - tot0) <= 1e-5 * abs(tot0), (f, tot0, tot)
    for f in ("bx", "by", "bz"):
        assert not g[f].any()


@pytest.mark.parametrize("emf", ["e0", "arith"])
def test_ppm_other_emf_schemes_fp64_bit_exact(emf):
    need_gpu()
    dims = (37, 29, 11)
    s = I.turbulence(dims, seed=59, kpeak=2.0, mach=0.9, b0=(0.15, -0.2, 0.25))
    l = s.pop("_l")
    print("ppm emf", emf, flush=True)
    g, o, gd, od, _ = run_both(s, dims, 3, l=l, per_step=True, recon="ppm", emf=emf,
                               integrator="rk3")
    assert bit_equal(g, o)
    assert gd == od


def test_ppm_with_uct_fp64_bit_exact():
    """PPM with the UCT-HLL edge solve (its face data reconstructed to the
    edges with PPM too), RK3: bit-identical to the oracle."""
    need_gpu()
    dims = (37, 29, 11)
    s = I.turbulence(dims, seed=61, kpeak=2.0, mach=0.9, b0=(0.2, 0.15, -0.25))
    l = s.pop("_l")
    print("ppm uct", flush=True)
    g, o, gd, od, _ = run_both(s, dims, 3, l=l, per_step=True, recon="ppm", emf="uct_hll",
                               integrator="rk3")
    assert bit_equal(g, o)
    assert gd == od
