"""GPU-test helpers: run the HIP library and the oracle on the same inputs."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O

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
                  cfl=0.3):
    nx, ny, nz = dims
    return O.Params(nx, ny, nz, *l, gamma=gamma, cfl=cfl,
                    riemann={"hlld": O.HLLD, "hll": O.HLL}[riemann],
                    integrator={"rk2": O.RK2, "euler": O.EULER}[integrator])


def run_both(state, dims, nsteps, l=(1.0, 1.0, 1.0), riemann="hlld", precision="fp64",
             integrator="rk2", per_step=False, **kw):
    """Advance the same input on the GPU and in the oracle; returns
    (gpu_state, oracle_state, gpu_dts, oracle_dts) with the dt_next sequence."""
    box = gpu_box(dims, l, precision=precision, riemann=riemann, integrator=integrator, **kw)
    box.set_state(state, 0.0, 0.0)
    orc = O.copy_state(state)
    p = oracle_params(dims, l, riemann, integrator)
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
