"""The C-ABI library loads and exports every function include/odf.h declares;
host-only calls (grid size, argument validation) behave without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2105_13611_amd import odf, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "odf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(odf_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(odf.LIB_PATH):
        from paper_2105_13611_amd import build
        build.build()
    return odf.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(odf.SIGNATURES), "binding signatures must cover the header"


def test_grid_points(lib):
    for (lf, ll, n) in [(300.0, 310.0, 16395), (8.9766, 10000.0, 3507864)]:
        lay = workload.Layout(lf, ll, 5e5, np.array([0, n], dtype=np.int64), np.array([1.0]))
        assert odf.grid_points(lay) == n
    bad = odf.OdfLayout(10.0, 5.0, 5e5, 0, None, 0, None)
    assert lib.odf_grid_points(C.byref(bad)) == -1


def _plan_args(w, **over):
    L = w.lines
    keep = dict(lam=odf._f64(L.lambda_nm), gf=odf._f64(L.log_gf), e=odf._f64(L.e_low_ev),
                sp=odf._i32(L.species), st=odf._i32(L.stage), gr=odf._f64(L.log_g_rad),
                gs=odf._f64(L.log_g_stark), gw=odf._f64(L.log_g_vdw),
                mass=odf._f64(w.species.mass_amu), chi=odf._f64(w.species.chi_ev),
                part=odf._f64(w.species.part_fn))
    keep.update(over)
    k = keep
    cl = odf.OdfLines(k["lam"].size, odf._ptr(k["lam"], odf._D), odf._ptr(k["gf"], odf._D),
                      odf._ptr(k["e"], odf._D), odf._ptr(k["sp"], odf._I32), odf._ptr(k["st"], odf._I32),
                      odf._ptr(k["gr"], odf._D), odf._ptr(k["gs"], odf._D), odf._ptr(k["gw"], odf._D))
    cs = odf.OdfSpecies(k["mass"].size, w.species.part_fn.shape[1], odf._ptr(k["mass"], odf._D),
                        odf._ptr(k["chi"], odf._D), odf._ptr(k["part"], odf._D))
    lay, lk = odf.make_layout(w.layout)
    keep["_lk"] = lk
    o = w.options
    opts = odf.OdfOptions(0, 0, o.cutoff, o.window_cap_doppler, o.pe_over_p, o.kappa_c_ref,
                          o.lambda_c_ref_nm, o.kappa_c_power, C.c_void_p(1), 1 << 20, None, 0, 0, 0)
    return cl, cs, lay, opts, keep


@pytest.mark.parametrize("case", ["species", "stage", "lambda", "edges", "frac", "cutoff", "workspace",
                                  "nan_gf", "output", "electrons", "pe_over_p"])
def test_plan_rejects_bad_arguments_before_touching_the_device(lib, case):
    w = workload.config(1, n_lines=50)
    over = {}
    if case == "species":
        sp = w.lines.species.copy(); sp[3] = 99; over["sp"] = odf._i32(sp)
    if case == "stage":
        st = w.lines.stage.copy(); st[0] = -1; over["st"] = odf._i32(st)
    if case == "lambda":
        lam = w.lines.lambda_nm.copy(); lam[5] = -1.0; over["lam"] = odf._f64(lam)
    if case == "nan_gf":
        gf = w.lines.log_gf.copy(); gf[7] = np.nan; over["gf"] = odf._f64(gf)
    cl, cs, lay, opts, keep = _plan_args(w, **over)
    if case == "edges":
        e = w.layout.bin_edges.copy(); e[3] = e[2]
        keep["e2"] = odf._i64(e); lay.bin_edges = odf._ptr(keep["e2"], odf._I64)
    if case == "frac":
        f = w.layout.step_frac.copy() * 1.01
        keep["f2"] = odf._f64(f); lay.step_frac = odf._ptr(keep["f2"], odf._D)
    if case == "cutoff":
        opts.cutoff = float("nan")
    if case == "workspace":
        opts.workspace = None
    if case == "output":
        opts.output = 2
    if case == "electrons":
        opts.electrons = -1
    if case == "pe_over_p":
        opts.pe_over_p = 1.5          # checked while the electron pressure is fixed
    h = C.c_void_p()
    rc = lib.odf_plan(C.byref(cl), C.byref(cs), C.byref(lay), C.byref(opts), C.byref(h))
    assert rc == odf.ODF_E_INVALID
    assert h.value is None
    assert len(lib.odf_last_error()) > 0


def test_null_arguments(lib):
    h = C.c_void_p()
    assert lib.odf_plan(None, None, None, None, C.byref(h)) == odf.ODF_E_INVALID
    assert lib.odf_plan_destroy(None) == odf.ODF_OK
    assert lib.odf_compute(None, None, None) == odf.ODF_E_INVALID
    assert lib.odf_submit(None, None, None) == odf.ODF_E_INVALID
    assert lib.odf_poll(None, 1, None) == odf.ODF_E_INVALID
    assert lib.odf_point_footprint(None) == -1
    assert lib.odf_stage_state(None, None, 0, None, None) == odf.ODF_E_INVALID
    assert lib.odf_debug_set_newton_limit(None, 5) == odf.ODF_E_INVALID
