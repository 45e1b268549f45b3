"""PPM reconstruction (Sec. 2.3; Colella & Woodward 1984 with the Colella &
Sekora 2008 extremum limiter) on the GPU against the FP64 oracle.

The stage kernel widens its LDS halo to three cells and its z-window to five
planes for PPM; these cases cross tile and z-chunk boundaries, wrap the
periodic halo more than once around a two-cell extent, and run every tile
shape.  FP64 must be bit-identical; FP32 is checked stage by stage against the
oracle's stage on the GPU's own input, to 1e-5 except where a PPM decision
within FP32 rounding of its threshold, taken the other way by the oracle, gives
the GPU's value (gpu_util.ppm_flip_check).
"""
import pytest

import numpy as np

from gpu_util import (bit_equal, check_fp32_ppm_cycles, gpu_box, max_rel, need_gpu, oracle_params,
                      run_both)
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


def _check_ppm_fp32(s, dims, ncycles, **kw):
    """FP32 PPM one RK3 cycle at a time, every stage against the oracle's stage
    on the GPU's own input (gpu_util.check_fp32_ppm_cycles): 1e-5 everywhere,
    except cells that near PPM decisions taken the other way (R21) or E^c ties
    (R16) explain."""
    box = gpu_box(dims, precision="fp32", recon="ppm", integrator="rk3", **kw)
    box.set_state(s)
    p = oracle_params(dims, riemann=kw.get("riemann", "hlld"), integrator="rk3",
                      emf=kw.get("emf", "ec"), recon="ppm")
    tot = check_fp32_ppm_cycles(box, p, ncycles)
    box.close()
    return tot


@pytest.mark.parametrize("riemann", ["hlld", "hll"])
def test_ppm_fp32_stagewise(riemann):
    """FP32 PPM on Orszag-Tang 32^3, 5 RK3 cycles, stage by stage (R21)."""
    need_gpu()
    s = I.to_float32_exact(I.orszag_tang(32))
    print("ppm fp32", riemann, flush=True)
    tot = _check_ppm_fp32(s, (32, 32, 32), 5, riemann=riemann)
    print("ppm fp32", riemann, tot)
    assert tot["unexplained"] == 0


@pytest.mark.parametrize("emf", ["e0", "arith", "uct_hll"])
def test_ppm_fp32_other_emf_schemes(emf):
    """FP32 PPM with the EMF schemes that take no upwind decision, on the same
    Orszag-Tang run, stage by stage (R21)."""
    need_gpu()
    s = I.to_float32_exact(I.orszag_tang(32))
    print("ppm fp32", emf, flush=True)
    tot = _check_ppm_fp32(s, (32, 32, 32), 4, emf=emf)
    print("ppm fp32", emf, tot)
    assert tot["unexplained"] == 0


def test_ppm_sedov_hllc_fp32():
    """FP32 PPM on the Sedov-Taylor blast, 6 RK3 cycles, every stage against the
    oracle's stage on the GPU's own input (R21: the blast front puts PPM
    decisions within FP32 rounding of their thresholds, and cells there may take
    the other outcome); and what rounding cannot change: finite, positive
    density and pressure, mass and energy conserved to FP32 rounding, the field
    exactly zero."""
    need_gpu()
    n = 32
    s = I.to_float32_exact(I.sedov(n))
    print("ppm sedov hllc fp32 rk3", flush=True)
    box = gpu_box((n, n, n), precision="fp32", riemann="hllc", recon="ppm", integrator="rk3")
    box.set_state(s)
    p = oracle_params((n, n, n), riemann="hllc", integrator="rk3", recon="ppm")
    tot = check_fp32_ppm_cycles(box, p, 6)
    print("ppm sedov fp32", tot)
    g, _, _, rc = box.get_state_numpy()
    box.close()
    assert rc == 0 and tot["unexplained"] == 0
    ke = 0.5 * (g["mx"] ** 2 + g["my"] ** 2 + g["mz"] ** 2) / g["rho"]
    pr = (5.0 / 3.0 - 1.0) * (g["en"] - ke)
    assert np.isfinite(pr).all() and g["rho"].min() > 0 and pr.min() > 0
    for f in ("rho", "en"):
        tot0, tot1 = float(np.sum(s[f])), float(np.sum(g[f]))
        assert abs(tot1 - tot0) <= 1e-5 * abs(tot0), (f, tot0, tot1)
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
