"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2105_13611_amd.prof_summary stats --csv <run_kernel_stats.csv>
      --command "<profiled command>" --title "..." --out profiles/<name>.md
  python -m paper_2105_13611_amd.prof_summary traffic --fetch <counter csv>
      --write <counter csv> --copy-mb 1024 --kernel k_voigt32
      --command "<profiled command>" --out profiles/<name>.md
  python -m paper_2105_13611_amd.prof_summary passes --fetch <counter csv>
      --write <counter csv> --trace <run_kernel_trace.csv> --copy-mb 1024
      --command "<profiled commands>" --out profiles/<name>.md
  python -m paper_2105_13611_amd.prof_summary flops --csv <counter csv>
      --bench-log <the profiled run's output> --kernel k_voigt32
      --command "<profiled command>" --out profiles/<name>.md
  python -m paper_2105_13611_amd.prof_summary issue --csv <counter csv>
      --kernel k_voigt32 --command "<profiled command>" --out profiles/<name>.md

`traffic` scales each kernel's FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
by the ratio of the bytes a plain elementwise copy of known size moves to what
the same counter reads for it, and records the hash of the Voigt kernel
sources, so that the benchmark can tell whether the figure still applies.
"""
import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in ("k_voigt.hip", "odf_internal.h"):
        with open(os.path.join(ROOT, "paper_2105_13611_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name):
    m = re.search(r"(k_\w+|\w*elementwise\w*|\w*copy\w*)", name)
    return m.group(1) if m else name[:60]


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {args.title}", "", "Command (run from the repository root on one MI355X):", "",
             "```", args.command, "```", "",
             "| kernel | calls | total ms | avg ms | min ms | max ms | % |", "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e6:.3f} | {float(r['MinNs']) / 1e6:.3f} | "
                     f"{float(r['MaxNs']) / 1e6:.3f} | {100 * float(r['TotalDurationNs']) / total:.1f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")


def per_dispatch(path, counter):
    """{dispatch id: (kernel name, value)} for one counter."""
    out = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        name, v = out.get(d, (r["Kernel_Name"], 0.0))
        out[d] = (name, v + float(r["Counter_Value"]))
    return out


def traffic(args):
    copy_bytes = args.copy_mb << 20
    res = {}
    for counter, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        d = per_dispatch(path, counter)
        copies = [v for n, v in d.values() if "elementwise" in n or "mul" in short_name(n)]
        # the calibration copies are the largest elementwise dispatches
        copies = sorted(copies)[-3:]
        kib = sum(copies) / len(copies)
        factor = copy_bytes / (kib * 1024.0)
        ker = [v for n, v in d.values() if args.kernel in n]
        res[counter] = dict(copy_kib=kib, factor=factor, dispatches=len(ker),
                            bytes_per_launch=factor * 1024.0 * sum(ker) / len(ker))
    hbm = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    summary = dict(kernel=args.kernel, source_sha256=kernel_sources_sha256(),
                   hbm_bytes_per_launch=hbm,
                   fetch_bytes_per_launch=res["FETCH_SIZE"]["bytes_per_launch"],
                   write_bytes_per_launch=res["WRITE_SIZE"]["bytes_per_launch"],
                   launches=res["FETCH_SIZE"]["dispatches"],
                   copy_bytes=copy_bytes, fetch_factor=res["FETCH_SIZE"]["factor"],
                   write_factor=res["WRITE_SIZE"]["factor"],
                   copy_fetch_kib=res["FETCH_SIZE"]["copy_kib"], copy_write_kib=res["WRITE_SIZE"]["copy_kib"])
    if args.bench_log:
        # per Voigt sample, so that a run batched differently can scale it
        j = json.loads([l for l in open(args.bench_log) if l.startswith("{")][-1])
        samples = j["voigt_samples_per_point"] * j["config"]["points"] * j["steps"]
        summary["voigt_samples"] = samples
        summary["hbm_bytes_per_sample"] = hbm * summary["launches"] / samples
    lines = [f"# HBM traffic of {args.kernel}", "", args.title, "",
             "Commands (run from the repository root on one MI355X, one counter per pass):", "",
             "```", args.command, "```", "",
             f"- calibration: an elementwise copy of {args.copy_mb} MiB reads "
             f"{summary['copy_fetch_kib']:.0f} KiB (FETCH_SIZE) and writes {summary['copy_write_kib']:.0f} KiB "
             f"(WRITE_SIZE); factors {summary['fetch_factor']:.4f} and {summary['write_factor']:.4f}",
             f"- {args.kernel}: {summary['launches']} launches, "
             f"{summary['fetch_bytes_per_launch'] / 1e9:.3f} GB read and "
             f"{summary['write_bytes_per_launch'] / 1e9:.3f} GB written per launch (calibrated)"
             + (f"; {summary['hbm_bytes_per_sample']:.4f} B per Voigt sample" if "hbm_bytes_per_sample" in summary else ""),
             "", "```json", json.dumps(summary, indent=1), "```", ""]
    open(args.out, "w").write("\n".join(lines))


def passes(args):
    """HBM bytes (calibrated FETCH_SIZE + WRITE_SIZE) and the rate over the
    traced durations of every engine kernel of one profiled table run."""
    copy_bytes = args.copy_mb << 20
    per = {}
    factors = {}
    for counter, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        d = per_dispatch(path, counter)
        copies = sorted(v for n, v in d.values() if "elementwise" in n or "mul" in short_name(n))[-3:]
        factors[counter] = copy_bytes / (sum(copies) / len(copies) * 1024.0)
        for n, v in d.values():
            if "odf::" not in n or not short_name(n).startswith("k_"):
                continue
            e = per.setdefault(short_name(n), {"FETCH_SIZE": [], "WRITE_SIZE": []})
            e[counter].append(factors[counter] * 1024.0 * v)
    dur = defaultdict(list)
    for r in csv.DictReader(open(args.trace)):
        n = r["Kernel_Name"]
        if "odf::" in n and short_name(n).startswith("k_"):
            dur[short_name(n)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    lines = [f"# HBM traffic of every pass: {args.title}", "",
             "Commands (run from the repository root on one MI355X, one counter per pass):", "",
             "```", args.command, "```", "",
             f"- calibration factors (elementwise copy of {args.copy_mb} MiB): FETCH_SIZE "
             f"{factors['FETCH_SIZE']:.4f}, WRITE_SIZE {factors['WRITE_SIZE']:.4f}",
             "- durations are the kernel trace's per-dispatch times of the same table in another run; "
             "kernels of the three internal streams overlap, so a dispatch's time includes time it "
             "shares the GPU and the rates are lower bounds", "",
             "| kernel | launches | GB read per launch | GB written per launch | avg ms (trace) | GB/s | fraction of 8 TB/s |",
             "|---|---|---|---|---|---|---|"]
    for k in sorted(per, key=lambda k: -sum(per[k]["FETCH_SIZE"])):
        f, w = per[k]["FETCH_SIZE"], per[k]["WRITE_SIZE"]
        n = max(len(f), 1)
        rd, wr = sum(f) / n, (sum(w) / len(w) if w else 0.0)
        t = sum(dur[k]) / len(dur[k]) if dur.get(k) else 0.0
        rate = (rd + wr) / t / 1e9 if t > 0 else 0.0
        lines.append(f"| {k} | {n} | {rd / 1e9:.3f} | {wr / 1e9:.3f} | {t * 1e3:.3f} | {rate:.1f} | {rate / 8000.0:.4f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")


def flops(args):
    """Executed floating-point operations of one kernel from the VALU counters
    (wave instructions x 64 lanes; FMA = 2), per Voigt sample of the profiled
    run (the samples come from that run's benchmark line)."""
    counters = defaultdict(float)
    launches = set()
    for r in csv.DictReader(open(args.csv)):
        if args.kernel in r["Kernel_Name"]:
            counters[r["Counter_Name"]] += float(r["Counter_Value"])
            launches.add(r["Dispatch_Id"])
    line = [l for l in open(args.bench_log) if l.startswith("{")][-1]
    j = json.loads(line)
    samples = j["voigt_samples_per_point"] * j["config"]["points"] * j["steps"]
    suffix = "F32" if "32" in args.kernel else "F64"
    weight = {f"SQ_INSTS_VALU_ADD_{suffix}": 1, f"SQ_INSTS_VALU_MUL_{suffix}": 1,
              f"SQ_INSTS_VALU_FMA_{suffix}": 2, f"SQ_INSTS_VALU_TRANS_{suffix}": 1}
    flop = sum(64.0 * counters[k] * w for k, w in weight.items())
    per_sample = flop / samples
    rate = per_sample * j["voigt_samples_per_s"] / 1e12 if "voigt_samples_per_s" in j else None
    lines = [f"# Executed {suffix} operations of {args.kernel}", "", args.title, "",
             "Command (run from the repository root on one MI355X):", "", "```", args.command, "```", "",
             "| counter | wave instructions | per Voigt sample (x64 lanes) |", "|---|---|---|"]
    for k in sorted(counters):
        lines.append(f"| {k} | {counters[k]:.4e} | {64.0 * counters[k] / samples:.3f} |")
    lines += ["", f"- {len(launches)} launches, {samples:.4e} Voigt samples",
              f"- executed {suffix} FLOP per sample (FMA = 2, all 64 lanes counted): {per_sample:.2f}",
              f"- at the profiled run's sample rate ({j.get('voigt_samples_per_s', 0):.4e}/s, which the "
              f"profiler slows): {rate:.2f} TFLOP/s" if rate else ""]
    summary = dict(kernel=args.kernel, source_sha256=kernel_sources_sha256(),
                   executed_flop_per_sample=per_sample, voigt_samples=samples, launches=len(launches))
    lines += ["", "```json", json.dumps(summary, indent=1), "```"]
    open(args.out, "w").write("\n".join(lines) + "\n")


# MI355X: 8 XCDs of 32 compute units, 4 SIMDs per compute unit
XCDS = 8
SIMDS = 256 * 4


def issue(args):
    """How busy the SIMDs' vector issue is over one kernel's dispatches.

    GRBM_GUI_ACTIVE counts the cycles the GPU is busy, once per XCD, so over
    a dispatch it sums to 8 x the dispatch's cycles; each SIMD then has that
    many cycles / 8 to issue in.  A wave64 VALU instruction occupies its
    SIMD for at least 4 cycles (16 lanes per cycle), so
        VALU busy >= 4 SQ_INSTS_VALU / (SIMDs x GRBM_GUI_ACTIVE / 8)
    (a lower bound: transcendental and FP64 instructions take longer)."""
    counters = defaultdict(float)
    launches = set()
    for r in csv.DictReader(open(args.csv)):
        if args.kernel in r["Kernel_Name"]:
            counters[r["Counter_Name"]] += float(r["Counter_Value"])
            launches.add(r["Dispatch_Id"])
    g = counters.get("GRBM_GUI_ACTIVE", 0.0)
    simd_cycles = SIMDS * g / XCDS
    lines = [f"# Issue counters of {args.kernel}: {args.title}", "",
             "Command (run from the repository root on one MI355X; one pass):", "",
             "```", args.command, "```", "",
             f"Sums over the {len(launches)} {args.kernel} dispatches of the run:", "",
             "| counter | sum |", "|---|---|"]
    for k in sorted(counters):
        lines.append(f"| {k} | {counters[k]:.4e} |")
    summary = dict(kernel=args.kernel, source_sha256=kernel_sources_sha256(), launches=len(launches))
    lines.append("")
    if g > 0 and "SQ_INSTS_VALU" in counters:
        busy = 4.0 * counters["SQ_INSTS_VALU"] / simd_cycles
        summary["valu_issue_busy_lower_bound"] = busy
        lines.append(f"- GPU busy {g / XCDS:.4e} cycles (GRBM_GUI_ACTIVE / {XCDS} XCDs); each of the "
                     f"{SIMDS} SIMDs issues VALU instructions in at least {100 * busy:.1f} % of them "
                     "(4 cycles per wave64 VALU instruction)")
        if "SQ_INSTS_VALU_TRANS_F32" in counters:
            t = counters["SQ_INSTS_VALU_TRANS_F32"] / counters["SQ_INSTS_VALU"]
            summary["trans_fraction"] = t
            lines.append(f"- {100 * t:.1f} % of the VALU instructions are transcendental (FP32)")
    if "SQ_WAVE_CYCLES" in counters:
        w = counters["SQ_WAVE_CYCLES"]
        for k, what in (("SQ_ACTIVE_INST_VALU", "issues VALU"), ("SQ_ACTIVE_INST_SCA", "issues scalar"),
                        ("SQ_WAIT_INST_ANY", "waits on a dependency or memory")):
            if k in counters:
                lines.append(f"- a wave {what} in {100 * counters[k] / w:.1f} % of its cycles")
    if "SQ_INSTS_SALU" in counters and "SQ_INSTS_VALU" in counters:
        lines.append(f"- {counters['SQ_INSTS_SALU'] / counters['SQ_INSTS_VALU']:.2f} scalar instructions "
                     "per VALU instruction")
    if "SQ_INSTS_LDS" in counters and "SQ_INSTS_VALU" in counters:
        lines.append(f"- {counters['SQ_INSTS_LDS'] / counters['SQ_INSTS_VALU']:.3f} LDS instructions "
                     "per VALU instruction")
    lines += ["", "```json", json.dumps(summary, indent=1), "```"]
    open(args.out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--csv", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--title", default="Kernel trace")
    a.add_argument("--out", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-mb", type=int, required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--bench-log", default="", help="benchmark line of the FETCH_SIZE run (samples)")
    b.add_argument("--command", required=True)
    b.add_argument("--title", default="")
    b.add_argument("--out", required=True)
    e = sub.add_parser("passes")
    e.add_argument("--fetch", required=True)
    e.add_argument("--write", required=True)
    e.add_argument("--trace", required=True)
    e.add_argument("--copy-mb", type=int, required=True)
    e.add_argument("--command", required=True)
    e.add_argument("--title", default="")
    e.add_argument("--out", required=True)
    c = sub.add_parser("flops")
    c.add_argument("--csv", required=True)
    c.add_argument("--bench-log", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--out", required=True)
    i = sub.add_parser("issue")
    i.add_argument("--csv", required=True)
    i.add_argument("--kernel", required=True)
    i.add_argument("--command", required=True)
    i.add_argument("--title", default="")
    i.add_argument("--out", required=True)
    args = ap.parse_args()
    {"stats": stats, "traffic": traffic, "passes": passes, "flops": flops, "issue": issue}[args.cmd](args)


if __name__ == "__main__":
    main()
