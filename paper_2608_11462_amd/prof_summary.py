"""Summaries of rocprofv3 runs of bench.py for profiles/ (text only).

    python -m paper_2608_11462_amd.prof_summary kernels <dir> <out.md> "<command>"
    python -m paper_2608_11462_amd.prof_summary traffic <fetch_dir> <write_dir> <out.md> \
        "<fetch command>" "<write command>"
    python -m paper_2608_11462_amd.prof_summary sq <out.md> <dir> "<command>" [<dir> "<command>" ...]

`kernels` reads the `*_kernel_stats.csv` and `*_kernel_trace.csv` files that
`rocprofv3 --kernel-trace --stats --output-format csv` writes and tabulates
calls, total and average duration, share, VGPRs and LDS bytes per kernel.

`sq` reads the `*_counter_collection.csv` files of one or more `--pmc` passes of
SQ counters and tabulates, for the step's main kernels, each counter per
dispatch (summed over the dispatch's wavefronts) and per wavefront.

`traffic` reads the `*_counter_collection.csv` files of two `--pmc` passes
(FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), scales them by what the same
counters read for the calibration copy of `bench.py --copy-calibration` (one
elementwise kernel reading and writing 1 GiB), tabulates per-dispatch bytes,
and writes profiles/traffic_<kernel>_large_tps.json for the kernels whose
rooflines bench.py reports (with the hash of the source file each comes
from, so stale counters are not reported).
"""
from __future__ import annotations

import csv
import hashlib
import json
import sys
from collections import defaultdict
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2608_11462_amd" / "csrc"
GIB_KIB = 1 << 20  # the calibration copy moves 1 GiB each way

# roofline kernels: bench name -> (kernel-name prefix in the trace, source file)
ROOF = {
    "leaf_eval": ("kf_leaf_eval<double, double, 2>", "fmm_log.hip"),
    "m2l": ("kf_m2l_mfma<27>", "fmm_log.hip"),
    "vecchia_factor": ("k_factor<32>", "vecchia.hip"),
    "precond_u": ("kf_apply_u", "forest.hip"),
    "precond_ut": ("kf_apply_ut", "forest.hip"),
}


def _rows(d: Path, suffix: str):
    for f in sorted(Path(d).rglob(f"*{suffix}")):
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def _short(name: str) -> str:
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    name = name.replace("phs::", "").replace("(anonymous namespace)::", "")
    cut = name.find("(")
    return name[:cut] if cut > 0 else name


def source_sha(name: str) -> str:
    return hashlib.sha256((CSRC / name).read_bytes()).hexdigest()[:16]


def kernels(d: str, out: str, command: str) -> None:
    stats = list(_rows(Path(d), "_kernel_stats.csv"))
    meta = {}
    for r in _rows(Path(d), "_kernel_trace.csv"):
        meta.setdefault(_short(r.get("Kernel_Name", "")),
                        (r.get("VGPR_Count", ""), r.get("LDS_Block_Size", "")))
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel trace: n=2^20 thin-plate solve (large_tps), FP64 step", "",
             "Command (from the repository root, on one MI355X):", "", "```", command, "```", "",
             "Summary of the `*_kernel_stats.csv` written by rocprofv3 (durations in "
             "microseconds), with VGPRs and LDS bytes from the kernel trace:", "",
             "| kernel | calls | total us | avg us | % | VGPRs | LDS B |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in stats[:30]:
        nm = _short(r["Name"])
        vg, lds = meta.get(nm, ("", ""))
        lines.append(f"| `{nm}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.0f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} | "
                     f"{vg} | {lds} |")
    Path(out).write_text("\n".join(lines) + "\n")


def _per_dispatch(d: Path, counter: str):
    tot, cnt = defaultdict(float), defaultdict(int)
    for r in _rows(d, "_counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        nm = _short(r["Kernel_Name"])
        tot[nm] += float(r["Counter_Value"])
        cnt[nm] += 1
    return {k: (tot[k] / cnt[k], cnt[k]) for k in tot}


def traffic(fetch_dir: str, write_dir: str, out: str, fcmd: str, wcmd: str) -> None:
    fe = _per_dispatch(Path(fetch_dir), "FETCH_SIZE")
    wr = _per_dispatch(Path(write_dir), "WRITE_SIZE")
    cal = [k for k in fe if "mul" in k.lower() and "elementwise" in k.lower()]
    cal_k = max(cal, key=lambda k: fe[k][0]) if cal else None
    fs = GIB_KIB / fe[cal_k][0] if cal_k else 1.0
    ws = GIB_KIB / wr[cal_k][0] if cal_k and cal_k in wr else 1.0
    lines = ["# HBM traffic per dispatch: n=2^20 thin-plate solve (large_tps), FP64", "",
             "Commands (two passes, one counter each):", "", "```", fcmd, wcmd, "```", "",
             f"Calibration: `--copy-calibration` runs one elementwise kernel reading 1 GiB and "
             f"writing 1 GiB (`{cal_k}`). FETCH_SIZE read {fe[cal_k][0]:.0f} KiB and WRITE_SIZE "
             f"{wr.get(cal_k, (0, 0))[0]:.0f} KiB for it, so fetches are scaled by {fs:.3f} and "
             f"writes by {ws:.3f} below." if cal_k else "No calibration kernel found: unscaled.",
             "Values are per-dispatch averages of the counter collection.", "",
             "| kernel | dispatches | fetch MB/dispatch (scaled) | write MB/dispatch (scaled) |",
             "|---|---:|---:|---:|"]
    order = sorted(fe, key=lambda k: -(fe[k][0] * fs + wr.get(k, (0, 0))[0] * ws))
    for k in order:
        if k == cal_k:
            continue
        f_mb = fe[k][0] * fs * 1024 / 1e6
        w_mb = wr.get(k, (0, 0))[0] * ws * 1024 / 1e6
        if f_mb + w_mb < 0.05:
            continue
        lines.append(f"| `{k}` | {fe[k][1]} | {f_mb:.1f} | {w_mb:.1f} |")
    Path(out).write_text("\n".join(lines) + "\n")
    for bench_name, (prefix, src) in ROOF.items():
        if prefix not in fe:
            continue
        fb = fe[prefix][0] * fs * 1024
        wb = wr.get(prefix, (0, 0))[0] * ws * 1024
        (Path(out).parent / f"traffic_{bench_name}_large_tps.json").write_text(json.dumps({
            "kernel": prefix, "workload": "large_tps", "source": src,
            "source_sha": source_sha(src), "fetch_bytes_per_launch": round(fb),
            "write_bytes_per_launch": round(wb), "bytes_per_launch": round(fb + wb),
            "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
            "commands": [fcmd, wcmd]}, indent=1) + "\n")


SQ_KERNELS = ["kf_leaf_eval<double, double, 2>", "kf_m2l_mfma<27>", "k_factor<32>", "k_knn<2>",
              "kf_apply_u", "kf_apply_ut"]


def sq(out: str, passes) -> None:
    """passes: [(dir, command), ...]; one table row per kernel of SQ_KERNELS."""
    vals = defaultdict(dict)
    counters = []
    for d, _ in passes:
        tot, cnt = defaultdict(float), defaultdict(int)
        for r in _rows(Path(d), "_counter_collection.csv"):
            key = (_short(r["Kernel_Name"]), r["Counter_Name"])
            tot[key] += float(r["Counter_Value"])
            cnt[key] += 1
        for (k, c), v in tot.items():
            if c not in counters:
                counters.append(c)
            vals[k][c] = v / cnt[(k, c)]  # per dispatch (its records are per dispatch)
    lines = ["# SQ counters per dispatch: n=2^20 thin-plate solve (large_tps), FP64", "",
             "Commands (one pass per counter set, from the repository root):", "", "```"]
    lines += [c for _, c in passes]
    lines += ["```", "",
              "Each value is the counter summed over one dispatch's wavefronts, averaged over "
              "the dispatches of the run; `/wave` divides by `SQ_WAVES` where that was "
              "collected.", ""]
    cols = [c for c in counters]
    lines.append("| kernel | " + " | ".join(cols) + " |")
    lines.append("|---|" + "---:|" * len(cols))
    for k in SQ_KERNELS:
        if k not in vals:
            continue
        row = []
        for c in cols:
            v = vals[k].get(c)
            row.append("" if v is None else f"{v:.4g}")
        lines.append(f"| `{k}` | " + " | ".join(row) + " |")
    if any("SQ_WAVES" in vals[k] for k in vals):
        lines += ["", "Per wavefront:", "", "| kernel | " + " | ".join(c for c in cols if c != "SQ_WAVES") + " |",
                  "|---|" + "---:|" * (len(cols) - 1)]
        for k in SQ_KERNELS:
            if k not in vals or not vals[k].get("SQ_WAVES"):
                continue
            wv = vals[k]["SQ_WAVES"]
            lines.append(f"| `{k}` | " + " | ".join(
                "" if vals[k].get(c) is None else f"{vals[k][c] / wv:.4g}"
                for c in cols if c != "SQ_WAVES") + " |")
    Path(out).write_text("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        kernels(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "sq":
        rest = sys.argv[3:]
        sq(sys.argv[2], [(rest[i], rest[i + 1]) for i in range(0, len(rest), 2)])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6])
    else:
        raise SystemExit(__doc__)
