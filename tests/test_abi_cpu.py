"""The C-ABI library loads and exports every symbol include/mhd.h declares, and
rejects bad arguments before touching the GPU (runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mhd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    syms = declared_symbols()
    for s in ("mhd_create", "mhd_set_state", "mhd_step", "mhd_get_state", "mhd_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2304_13746_amd import _lib
    L = _lib.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(_lib.EXPORTED) == set(declared_symbols())


def test_workspace_bytes_and_argument_checks():
    from paper_2304_13746_amd import _lib
    from paper_2304_13746_amd.box import make_params
    L = _lib.lib()
    p = make_params(32, 32, 32, precision="fp64")
    n64 = L.mhd_workspace_bytes(C.byref(p))
    p32 = make_params(32, 32, 32, precision="fp32")
    n32 = L.mhd_workspace_bytes(C.byref(p32))
    # two 8-field state buffers dominate: 16 * N * word
    assert n64 >= 16 * 32 ** 3 * 8 and n32 >= 16 * 32 ** 3 * 4
    assert n64 - 16 * 32 ** 3 * 8 < 1 << 20
    bad = make_params(0, 32, 32)
    assert L.mhd_workspace_bytes(C.byref(bad)) == 0
    # extents up to 4096 cells per direction
    assert L.mhd_workspace_bytes(C.byref(make_params(4096, 2, 3))) > 0
    assert L.mhd_workspace_bytes(C.byref(make_params(4097, 2, 3))) == 0
    assert L.mhd_workspace_bytes(C.byref(make_params(2, 3, 4097))) == 0
    ctx = C.c_void_p()
    # invalid grid, gamma, cfl: rejected before any device call
    for kw in ({"nx": 0}, {"gamma": 1.0}, {"cfl": 1.0}, {"cfl": 0.0}):
        q = make_params(8, 8, 8)
        for k, v in kw.items():
            setattr(q, k, v)
        assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_INVALID_ARG
    q = make_params(8, 8, 8)
    q.emf = 7
    assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_UNSUPPORTED
    # PPM: every EMF scheme, both CT forms (the potential form in FP64)
    for kw in ({"recon": "ppm", "riemann": "hllc", "ct": "vecpot"},
               {"recon": "ppm", "ct": "vecpot", "precision": "fp32"}):
        q = make_params(8, 8, 8, **kw)
        assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_UNSUPPORTED, kw
    for kw in ({"recon": "ppm", "emf": "e0"}, {"recon": "ppm", "emf": "arith"},
               {"recon": "ppm", "ct": "vecpot"}, {"recon": "ppm", "emf": "uct_hll"}):
        q = make_params(8, 8, 8, **kw)
        assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_WORKSPACE, kw
    # UCT-HLL: MHD solvers, PLM or LimO3, face-field CT
    for kw in ({"emf": "uct_hll", "riemann": "hllc"},
               {"emf": "uct_hll", "ct": "vecpot", "precision": "fp32"}):
        q = make_params(8, 8, 8, **kw)
        assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_UNSUPPORTED, kw
    for kw in ({"recon": "ppm"}, {"recon": "ppm", "riemann": "hllc", "emf": "e0"},
               {"emf": "uct_hll"}, {"emf": "uct_hll", "riemann": "hll", "precision": "fp32"},
               {"emf": "uct_hll", "recon": "limo3"}, {"emf": "uct_hll", "ct": "vecpot"},
               {"emf": "e0", "ct": "vecpot"}, {"emf": "arith", "ct": "vecpot", "riemann": "hll"}):
        q = make_params(8, 8, 8, **kw)  # accepted up to the (missing) workspace
        assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_WORKSPACE, kw
    # UCT-HLL takes 15 more arrays of one field in the workspace, UCT-HLLD 21
    pu = make_params(32, 32, 32, precision="fp64", emf="uct_hll")
    assert L.mhd_workspace_bytes(C.byref(pu)) - n64 == 15 * 32 ** 3 * 8
    pu = make_params(32, 32, 32, precision="fp64", emf="uct_hlld")
    assert L.mhd_workspace_bytes(C.byref(pu)) - n64 == 21 * 32 ** 3 * 8
    # UCT-HLLD takes its coefficients from the HLLD solve
    for kw in ({"emf": "uct_hlld", "riemann": "hll"}, {"emf": "uct_hlld", "riemann": "hllc"},
               {"emf": "uct_hlld", "ct": "vecpot", "precision": "fp32"}):
        q = make_params(8, 8, 8, **kw)
        assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_UNSUPPORTED, kw
    for kw in ({"emf": "uct_hlld"}, {"emf": "uct_hlld", "precision": "fp32", "recon": "ppm"},
               {"emf": "uct_hlld", "ct": "vecpot", "recon": "limo3"}):
        q = make_params(8, 8, 8, **kw)
        assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_WORKSPACE, kw
    # no workspace / too small / misaligned
    q = make_params(8, 8, 8)
    assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_WORKSPACE
    q.workspace = 256
    q.workspace_bytes = 16
    assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_WORKSPACE
    q.workspace = 1024 + 8
    q.workspace_bytes = 1 << 40
    assert L.mhd_create(C.byref(q), C.byref(ctx)) == _lib.MHD_ERR_WORKSPACE
    assert L.mhd_create(None, C.byref(ctx)) == _lib.MHD_ERR_INVALID_ARG
    assert L.mhd_step(None, 1, 0.0) == _lib.MHD_ERR_INVALID_ARG
    assert L.mhd_destroy(None) == _lib.MHD_OK
    assert _lib.status_string(_lib.MHD_ERR_NONPHYSICAL).startswith("non-physical")


def test_launch_shape_and_tuner_argument_checks():
    from paper_2304_13746_amd import _lib
    L = _lib.lib()
    t, z = C.c_int(), C.c_int()
    assert L.mhd_set_launch(None, 0, 0) == _lib.MHD_ERR_INVALID_ARG
    assert L.mhd_get_launch(None, C.byref(t), C.byref(z)) == _lib.MHD_ERR_INVALID_ARG
    res = _lib.TuneResult()
    assert L.mhd_tune(None, 1, 3, None, C.byref(res)) == _lib.MHD_ERR_INVALID_ARG
    arr = (C.c_void_p * 1)(None)
    assert L.mhd_tune(arr, 1, 3, None, C.byref(res)) == _lib.MHD_ERR_INVALID_ARG
    assert L.mhd_tune(arr, 0, 3, None, C.byref(res)) == _lib.MHD_ERR_INVALID_ARG
