"""Host logic of bench.py (no GPU): roofline arithmetic on a synthetic result,
the counter-summary lookup, the stratified sample and the one-GPU guard."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
from paper_2105_13611_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _result():
    st = {k: dict(ms=0.0, busy_ms=0.0, launches=0) for k in ("point_state", "select", "scan", "emit", "odf")}
    st["voigt"] = dict(ms=400.0, busy_ms=300.0, launches=4)
    return dict(stage_ms=st, steps=2, stats=dict(voigt_samples=3.0e12),
                kernel_alone=dict(ms=50.0, busy_ms=50.0, launches=2, samples=2.0e11, points=64, batch_points=16))


def test_roofline_uses_the_average_launch_duration():
    r = bench.roofline(_result(), 10.0, "mixed")
    # 2 steps x 3e12 samples x 10 FLOP over 4 launches of 100 ms each
    assert abs(r["achieved"] - 6.0e13 / 0.4 / 1e12) < 1e-9
    assert r["peak"] == 157.3 and abs(r["frac"] - r["achieved"] / 157.3) < 1e-12
    # the union of the launch intervals is reported beside it
    assert abs(r["achieved_busy"] - 6.0e13 / 0.3 / 1e12) < 1e-9
    assert r["avg_launch_ms"] == 100.0 and r["busy_ms_per_launch"] == 75.0
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    c = r["ceiling_nonpacked"]
    assert abs(c["peak"] - 78.6432) < 1e-9 and abs(c["frac"] - r["achieved"] / c["peak"]) < 1e-12
    ka = r["kernel_alone"]
    assert abs(ka["achieved"] - 2.0e11 * 10.0 / 0.05 / 1e12) < 1e-9
    assert ka["avg_launch_ms"] == 25.0
    r64 = bench.roofline(_result(), 28.0, "fp64")
    assert r64["peak"] == 78.6 and "ceiling_nonpacked" not in r64


def test_nonpacked_ceiling_is_the_valu_rate():
    assert abs(bench.PEAK_VALU_TFLOPS - 78.6432) < 1e-9


def test_parity_block():
    ref = {3: dict(steps=np.array([[1.0, 2.0], [4.0, 8.0]]), near_tie=[False, True]),
           7: dict(steps=np.array([[1.0, 1.0], [2.0, 2.0]]), near_tie=[False, False])}
    got = {"mixed": {3: np.array([[1.0005, 2.0], [4.0, 8.0]]), 7: np.array([[1.0, 1.0], [2.0, 2.0]])},
           "fp64": {3: np.array([[1.0, 2.0], [4.0, 8.0 * (1 + 3e-9)]])}}
    pb = bench.parity_block(ref, [10, 20], got)
    m, f = pb["mixed"], pb["fp64"]
    assert m["pairs"] == 4 and abs(m["max_rel_err"] - 5e-4) < 1e-12 and m["within_tolerance"]
    assert abs(m["max_abs_dlog10_kappa"] - np.log10(1.0005)) < 1e-12
    assert m["bins_with_near_tie_decisions"] == 1 and m["max_rel_err_in_those"] == 0.0
    # point 7 was not in the FP64 leg's points: only point 3 counts
    assert f["pairs"] == 2 and abs(f["max_rel_err"] - 3e-9) < 1e-15 and not f["within_tolerance"]
    assert abs(f["max_rel_err_in_those"] - 3e-9) < 1e-15


def test_cpu_leg_keeps_the_oracle_steps():
    """The CPU leg on the small single-point workload: its kept steps are
    the oracle's ODF of those bins."""
    import oracle
    w = W.config(1, n_lines=300)
    base, ref, bins = bench.cpu_baseline(w, 2)
    assert base["kind"] == "oracle" and base["cores"] == 2 and base["value"] > 0
    # CPU_BINS evenly spaced bins, or every bin of a smaller layout (20 here)
    assert sorted(ref) == [0] and bins == list(range(min(bench.CPU_BINS, w.layout.n_bins)))
    steps, _, _ = oracle.odf_point(w.lines, w.species, w.species.abundance, float(w.points.T_K[0]),
                                   float(w.points.log10_P[0]), float(w.points.vturb_kms[0]), w.layout,
                                   w.options, bins)
    np.testing.assert_array_equal(ref[0]["steps"], steps)
    assert len(ref[0]["near_tie"]) == len(bins)


def test_traffic_summary_lookup():
    for prec in ("mixed", "fp64"):
        t = bench.traffic_per_launch(prec)
        path = os.path.join(ROOT, "profiles", f"voigt{32 if prec == 'mixed' else 64}_full_table_hbm_traffic.md")
        txt = open(path).read()
        d = json.loads(txt[txt.index("```json") + 7: txt.index("```", txt.index("```json") + 7)])
        if d["source_sha256"] == bench.kernel_sources_sha256():
            assert t == d["hbm_bytes_per_launch"] and t > 0
        else:
            assert t is None


def test_executed_flop_summary_lookup():
    for prec in ("mixed", "fp64"):
        e = bench.executed_flop_per_sample(prec)
        path = os.path.join(ROOT, "profiles", f"voigt{32 if prec == 'mixed' else 64}_full_table_valu_flops.md")
        txt = open(path).read()
        if "```json" not in txt:
            assert e is None
            continue
        d = json.loads(txt[txt.index("```json") + 7: txt.index("```", txt.index("```json") + 7)])
        if d["source_sha256"] == bench.kernel_sources_sha256():
            assert e == d["executed_flop_per_sample"] and e > 0
        else:
            assert e is None


def test_stratified_points_hold_the_corners():
    pts = W.dfsynthe_tp_grid((2.0,))
    idx = bench.stratified_points(pts, 16)
    assert len(idx) == 16 and len(set(idx.tolist())) == 16
    T, P = pts.T_K[idx], pts.log10_P[idx]
    for t, p in [(T.min(), P.min()), (pts.T_K.min(), pts.log10_P.max()),
                 (pts.T_K.max(), pts.log10_P.min()), (pts.T_K.max(), pts.log10_P.max())]:
        assert np.any((np.isclose(T, t)) & (np.isclose(P, p)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pretab_lattice_is_on_the_dfsynthe_grid():
    import numpy as np
    import bench
    from paper_2105_13611_amd import workload as W
    g = W.dfsynthe_tp_grid()
    lt = np.log10(2000.0) + (2.0 / 56.0) * np.arange(10, 14)
    pts = bench._lattice(lt, [0.0, 0.5, 1.0])
    assert pts.n_points == 12
    # every lattice node is a point of the 57 x 25 table
    for T, P in zip(pts.T_K, pts.log10_P):
        assert np.min(np.abs(g.T_K / T - 1.0) + np.abs(g.log10_P - P)) < 1e-12


def test_subbin_combination_matches_a_direct_reduction():
    # sub-bins built from 200 elementary sub-bins equal the ODF reduced
    # with those borders directly (the geometric mean of a union of
    # equal-width sub-bins is the geometric mean of their means)
    import numpy as np
    import bench
    import oracle
    rng = np.random.default_rng(4)
    for n in (1000, 1733):
        v = 10.0 ** rng.uniform(-2, 6, n)
        for mean in ("geometric", "arithmetic"):
            elem = oracle.odf_reduce_bin(v, np.full(bench.N_ELEMENTARY, 1.0 / bench.N_ELEMENTARY), mean)
            for bs in [(0.9,), (0.8, 0.95), (0.5, 0.85, 0.99)]:
                fr = np.diff(np.concatenate([[0.0], bs, [1.0]]))
                got = bench.combine_steps(elem, bs, mean)
                np.testing.assert_allclose(got, oracle.odf_reduce_bin(v, fr, mean), rtol=1e-12)


def test_slab_error_matches_the_oracle_slab():
    import numpy as np
    import bench
    import oracle
    rng = np.random.default_rng(8)
    P, B, n = 2, 3, 300
    fr = np.array([0.7, 0.25, 0.05])
    kc = rng.uniform(0.2, 0.8, B)
    vals = 10.0 ** rng.uniform(-3, 5, (P, B, n))
    steps = np.array([[oracle.odf_reduce_bin(vals[p, b], fr, "geometric") for b in range(B)] for p in range(P)])
    cols = bench.slab_columns(kc)
    fine_I = np.array([[oracle.slab_fine_intensity(vals[p, b], kc[b], cols[b]) for b in range(B)]
                       for p in range(P)])
    ref = max(abs(oracle.slab_odf_intensity(steps[p, b], fr, kc[b], cols[b])[c] / fine_I[p, b, c] - 1.0)
              for p in range(P) for b in range(B) for c in range(cols.shape[1]))
    assert bench.slab_odf_error(steps, fr, fine_I, kc, cols) == pytest.approx(ref, rel=1e-12)
    np.testing.assert_allclose(cols * kc[:, None], np.tile(bench.SLAB_TAU_C, (B, 1)), rtol=1e-15)
