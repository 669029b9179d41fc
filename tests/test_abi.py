"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and host-side validation returns the documented codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1201_3588_amd import mcrt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b((?:mcrt|pah)_\w+)\s*\(", txt, re.M)))


def test_every_declared_symbol_is_exported():
    L = mcrt.lib()
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        names += declared(h)
    assert "mcrt_run" in names and "mcrt_build_tables" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.mcrt_version() == 104


def good_desc():
    d = mcrt.Desc()
    d.precision, d.n_lambda, d.n_species, d.nb, d.max_level, d.K = 0, 8, 1, 4, 0, 16
    d.n_cells, d.n_nodes = 64, 0
    d.base_size, d.T_lo, d.T_hi = 1.0, 3.0, 5000.0
    d.n_theta, d.n_phi = 2, 1
    fake = C.c_void_p(0x1000)
    for f in ("lambda_um", "kabs", "ksca", "g", "kind", "base_map", "rho"):
        setattr(d, f, fake)
    return d


def test_descriptor_validation_codes():
    L = mcrt.lib()
    nb = C.c_uint64()
    assert L.mcrt_tables_bytes(C.byref(good_desc()), C.byref(nb)) == 0
    assert nb.value > 0 and nb.value % 256 == 0
    for field, val in [("n_lambda", 1), ("n_species", 0), ("K", 1), ("precision", 7), ("nb", 0),
                       ("max_level", 11), ("n_cells", 0), ("T_hi", 1.0), ("base_size", -1.0)]:
        d = good_desc()
        setattr(d, field, val)
        assert L.mcrt_tables_bytes(C.byref(d), C.byref(nb)) == -1, field
        ctx = C.c_void_p()
        assert L.mcrt_ctx_create(C.byref(d), C.byref(ctx)) == -1, field
        assert not ctx.value
    d = good_desc()
    d.rho = None
    assert L.mcrt_ctx_create(C.byref(d), C.byref(C.c_void_p())) == -1
    d = good_desc()
    d.n_nodes = 3        # nodes without subdivision levels
    assert L.mcrt_ctx_create(C.byref(d), C.byref(C.c_void_p())) == -1


def test_call_order_and_capacity_codes():
    L = mcrt.lib()
    ctx = C.c_void_p()
    assert L.mcrt_ctx_create(C.byref(good_desc()), C.byref(ctx)) == 0
    try:
        opts = mcrt.RunOpts()
        opts.n_total = 10
        t = mcrt.Tallies(C.c_void_p(0x1000), C.c_void_p(0x1000), None, C.c_void_p(0x1000))
        assert L.mcrt_run(ctx, 0, 10, C.byref(opts), C.byref(t), None) == -2
        assert b"before" in L.mcrt_last_error(ctx)
        assert L.mcrt_temperatures(ctx, C.c_void_p(0x1000), 10, C.c_void_p(0x1000), None) == -2
        src = mcrt.Source()
        src.lum, src.teff = 1.0, 5000.0
        assert L.mcrt_build_tables(ctx, C.byref(src), C.c_void_p(0x1000), 16, None) == -4
        src.teff = float("nan")
        assert L.mcrt_build_tables(ctx, C.byref(src), C.c_void_p(0x1000), 1 << 30, None) == -5
        src.teff, src.beam_on = 5000.0, 1
        src.beam = (C.c_double * 3)(1.0, 1.0, 0.0)
        assert L.mcrt_build_tables(ctx, C.byref(src), C.c_void_p(0x1000), 1 << 30, None) == -5
        lay = mcrt.TableLayout()
        assert L.mcrt_table_layout_get(ctx, C.byref(lay)) == 0
        assert lay.total > lay.scratch > lay.R > lay.E
    finally:
        L.mcrt_ctx_destroy(ctx)
    assert L.mcrt_ctx_create(C.byref(good_desc()), None) == -1


def test_pah_descriptor_limits():
    from paper_1201_3588_amd import pah
    L = pah.lib()
    fake = C.c_void_p(0x1000)
    nb = C.c_uint64()

    def desc(M, nl, nbands=17):
        d = pah.PahDesc()
        d.M, d.n_lambda, d.n_bands = M, nl, nbands
        d.T = d.U = d.lambda_um = d.cabs = d.cband = d.ccont = fake
        return d

    assert L.pah_tables_bytes(C.byref(desc(500, 200)), C.byref(nb)) == 0 and nb.value > 500 * 500 * 2
    assert L.pah_tables_bytes(C.byref(desc(2274, 200)), C.byref(nb)) == 0     # 6 M + 13 nl = 16244
    for M, nl in [(2, 200), (500, 1), (2275, 200), (500, 1500)]:
        assert L.pah_tables_bytes(C.byref(desc(M, nl)), C.byref(nb)) == -1, (M, nl)
        ctx = C.c_void_p()
        assert L.pah_ctx_create(C.byref(desc(M, nl)), C.byref(ctx)) == -1 and not ctx.value
    d = desc(500, 200)
    d.U = None
    assert L.pah_tables_bytes(C.byref(d), C.byref(nb)) == -1


def test_observer_validation_codes():
    L = mcrt.lib()
    ctx = C.c_void_p()
    assert L.mcrt_ctx_create(C.byref(good_desc()), C.byref(ctx)) == 0
    try:
        def obs(**kw):
            o = mcrt.Observers()
            o.n_obs, o.npix, o.n_img_lambda, o.half_width, o.cos_cone = 2, 16, 2, 1.0, 0.9
            o.img_lambda[0], o.img_lambda[1] = 0, 1
            o.dir[0][2], o.dir[1][0] = 1.0, 2.0
            for k, v in kw.items():
                setattr(o, k, v)
            return o
        assert L.mcrt_set_observers(ctx, C.byref(obs())) == 0
        for bad in [dict(n_obs=9), dict(n_obs=-1), dict(npix=0), dict(n_img_lambda=0), dict(n_img_lambda=9),
                    dict(half_width=0.0), dict(half_width=float("inf")), dict(cos_cone=0.0), dict(cos_cone=1.5)]:
            assert L.mcrt_set_observers(ctx, C.byref(obs(**bad))) == -1, bad
        o = obs()
        o.img_lambda[1] = 0                              # repeated bin
        assert L.mcrt_set_observers(ctx, C.byref(o)) == -1
        o = obs()
        o.img_lambda[1] = 10_000                         # beyond the wavelength grid
        assert L.mcrt_set_observers(ctx, C.byref(o)) == -1
        o = obs()
        o.dir[1][0] = 0.0                                # zero direction
        assert L.mcrt_set_observers(ctx, C.byref(o)) == -1
        assert L.mcrt_set_observers(ctx, C.byref(obs(n_obs=0))) == 0
        assert L.mcrt_set_observers(ctx, None) == -1
    finally:
        L.mcrt_ctx_destroy(ctx)
    assert L.mcrt_read_counters_sync(None, None, None) == -1


def test_deferred_tally_workspace_codes():
    L = mcrt.lib()
    nbytes = C.c_uint64()
    ctx = C.c_void_p()
    assert L.mcrt_ctx_create(C.byref(good_desc()), C.byref(ctx)) == 0
    try:
        assert L.mcrt_jrec_ws_bytes(ctx, 100, C.byref(nbytes)) == -1           # below one chunk
        assert L.mcrt_jrec_ws_bytes(ctx, (1 << 35) + 1, C.byref(nbytes)) == -1
        assert L.mcrt_jrec_ws_bytes(ctx, (1 << 33) + 4096, C.byref(nbytes)) == 0       # 64-bit offsets
        assert nbytes.value >= 16 * ((1 << 33) + 4096)
        assert L.mcrt_jrec_ws_bytes(ctx, 1 << 20, None) == -1
        assert L.mcrt_jrec_ws_bytes(ctx, 1 << 20, C.byref(nbytes)) == 0
        small = nbytes.value
        assert small >= 2 * 8 * (1 << 20) and small % 256 == 0                # two record buffers
        assert L.mcrt_jrec_ws_bytes(ctx, 1 << 22, C.byref(nbytes)) == 0
        assert nbytes.value - small >= 2 * 8 * ((1 << 22) - (1 << 20))
        # the workspace needs the path tally: TALLY_J off is rejected
        opts = mcrt.RunOpts()
        opts.n_total, opts.jrec_ws, opts.jrec_capacity = 10, C.c_void_p(0x1000), 1 << 20
        t = mcrt.Tallies(C.c_void_p(0x1000), C.c_void_p(0x1000), None, C.c_void_p(0x1000))
        assert L.mcrt_run(ctx, 0, 10, C.byref(opts), C.byref(t), None) == -2       # tables not built yet
    finally:
        L.mcrt_ctx_destroy(ctx)
    d = good_desc()
    d.max_level = 8                                                              # records hold 24-bit lengths
    d.n_nodes = 0
    ctx = C.c_void_p()
    assert L.mcrt_ctx_create(C.byref(d), C.byref(ctx)) == 0
    try:
        assert L.mcrt_jrec_ws_bytes(ctx, 1 << 20, C.byref(nbytes)) == -6
    finally:
        L.mcrt_ctx_destroy(ctx)
