"""Host checks of the rocprofv3 summary arithmetic on synthetic counter files."""
import csv
import json

from paper_2105_13611_amd import prof_summary as PS


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_issue_busy_from_grbm(tmp_path):
    """Two dispatches of 1e6 GPU cycles each (GRBM summed over 8 XCDs) in
    which every SIMD issues a VALU instruction every 8 cycles: busy 0.5."""
    rows = []
    for d in (1, 2):
        k = "odf::(anonymous namespace)::k_voigt32(...)"
        rows.append(dict(Dispatch_Id=d, Kernel_Name=k, Counter_Name="GRBM_GUI_ACTIVE", Counter_Value=8 * 1e6))
        rows.append(dict(Dispatch_Id=d, Kernel_Name=k, Counter_Name="SQ_INSTS_VALU",
                         Counter_Value=PS.SIMDS * 1e6 / 8))
        rows.append(dict(Dispatch_Id=d, Kernel_Name=k, Counter_Name="SQ_INSTS_VALU_TRANS_F32",
                         Counter_Value=PS.SIMDS * 1e6 / 80))
        rows.append(dict(Dispatch_Id=d, Kernel_Name="other_kernel", Counter_Name="SQ_INSTS_VALU", Counter_Value=1e12))
    src = tmp_path / "c.csv"
    _write(src, rows)
    out = tmp_path / "o.md"
    import sys
    argv = sys.argv
    try:
        sys.argv = ["x", "issue", "--csv", str(src), "--kernel", "k_voigt32", "--command", "cmd", "--out", str(out)]
        PS.main()
    finally:
        sys.argv = argv
    text = out.read_text()
    j = json.loads(text[text.index("```json") + 7:text.rindex("```")])
    assert j["launches"] == 2
    assert abs(j["valu_issue_busy_lower_bound"] - 0.5) < 1e-12
    assert abs(j["trans_fraction"] - 0.1) < 1e-12
