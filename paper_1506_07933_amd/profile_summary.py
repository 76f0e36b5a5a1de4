"""Summarise rocprofv3 output of bench.py runs into profiles/.

    python -m paper_1506_07933_amd.profile_summary \
        --trace out/trace --fetch out/pmc_fetch --write out/pmc_write \
        --copy-fetch out/pmc_copy_fetch --copy-write out/pmc_copy_write \
        --passes z_contig,y_strided,x_strided --title "..." --command "..." --out profiles/x.md

The kernel trace gives per-dispatch durations; dispatches of the transform's
kernels are assigned to passes in launch order (the pass list repeats once per
transform).  FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled by what the
same counters read for a plain device copy of known size (bench.py --mode
copy), and the per-pass HBM bytes are written to profiles/traffic.json with a
hash of the kernel sources, so the benchmark can drop them once the kernels
change.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys


def _csv(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def _fft_dispatches(rows, skip=("twiddles", "k_copy", "k_tile_copy")):
    """The transform's own dispatches (library kernels other than the twiddle
    generator), in launch order."""
    rows = [r for r in rows if "mifft::k_" in r["Kernel_Name"]
            and not any(s in r["Kernel_Name"] for s in skip)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    return rows


def _per_pass(rows, npass):
    groups = [[] for _ in range(npass)]
    for i, r in enumerate(rows):
        groups[i % npass].append(r)
    return groups


def copy_scale(fetch_dir, write_dir, copy_bytes=1 << 30):
    f = [float(r["Counter_Value"]) for r in _csv(fetch_dir, "counter_collection.csv")
         if "copyBuffer" in r["Kernel_Name"]]
    w = [float(r["Counter_Value"]) for r in _csv(write_dir, "counter_collection.csv")
         if "copyBuffer" in r["Kernel_Name"]]
    kib = copy_bytes / 1024.0
    return kib / statistics.mean(f), kib / statistics.mean(w), statistics.mean(f), statistics.mean(w)


def stats_table(trace_dir: str, title: str, command: str, note: str = "") -> str:
    """Markdown table of a rocprofv3 --stats kernel summary (every kernel)."""
    rows = _csv(trace_dir, "kernel_stats.csv")
    lines = ["# " + title, "", "Command:", "", "    " + command, ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | calls | mean us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %.1f%% |" % (
            r["Name"].split("(")[0], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(lines) + "\n"


def kernels_table(trace_dir, fetch_dir, write_dir, copy_fetch, copy_write, alg, title, command, counter_command,
                  note=""):
    """Per-kernel table of one workload: mean duration (kernel trace), mean
    FETCH_SIZE / WRITE_SIZE per dispatch scaled by the plain-copy factors, and
    for kernels with a known algorithmic byte count per dispatch (`alg`:
    name fragment -> bytes) the ratio counter / algorithmic and the
    algorithmic rate.  Returns (markdown, {kernel: traffic entry})."""
    trace = _csv(trace_dir, "kernel_trace.csv")
    sf, sw, cf, cw = copy_scale(copy_fetch, copy_write)
    fr = _csv(fetch_dir, "counter_collection.csv")
    wr = _csv(write_dir, "counter_collection.csv")

    def short(name):
        return name.split("(")[0].replace("void ", "")

    def grid(r):
        return r.get("Grid_Size") or r.get("Grid_Size_X") or ""

    # a kernel launched with more than one grid (e.g. the fused spectral pass
    # over the main array and over the Nyquist plane) gets one row per grid
    grids = {}
    for r in trace:
        if "mifft::k_" in r["Kernel_Name"]:
            grids.setdefault(short(r["Kernel_Name"]), set()).add(grid(r))

    def name_of(r):
        k = short(r["Kernel_Name"])
        return "%s [grid %s]" % (k, grid(r)) if len(grids.get(k, ())) > 1 else k

    def by_kernel(rows, key):
        d = {}
        for r in rows:
            if "mifft::k_" not in r["Kernel_Name"]:
                continue
            d.setdefault(name_of(r), []).append(key(r))
        return d

    dur = by_kernel(trace, lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    fk = by_kernel(fr, lambda r: float(r["Counter_Value"]))
    wk = by_kernel(wr, lambda r: float(r["Counter_Value"]))
    lines = ["# " + title, "", "Command (kernel trace):", "", "    " + command, "",
             "Counters (separate runs, `--pmc FETCH_SIZE` then `--pmc WRITE_SIZE`):", "", "    " + counter_command, "",
             "Scale: a plain 1 GiB device copy reads FETCH_SIZE = %.1f KiB and WRITE_SIZE = %.1f KiB, so FETCH_SIZE "
             "is multiplied by %.4f and WRITE_SIZE by %.4f." % (cf, cw, sf, sw), ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | dispatches | mean us | HBM bytes / dispatch (counters) | algorithmic bytes | counter / alg "
              "| alg GB/s | of 8 TB/s |", "|---|---|---|---|---|---|---|---|"]
    traffic = {}
    for k in sorted(dur, key=lambda k: -sum(dur[k])):
        mean = statistics.mean(dur[k])
        hbm = None
        if k in fk and k in wk:
            hbm = (statistics.mean(fk[k]) * sf + statistics.mean(wk[k]) * sw) * 1024.0
        a = next((v for frag, v in alg.items() if frag in k), None)
        cells = ["`%s`" % k, str(len(dur[k])), "%.1f" % mean, "%.4g" % hbm if hbm else "-",
                 "%.4g" % a if a else "-", "%.4f" % (hbm / a) if (hbm and a) else "-",
                 "%.0f" % (a / (mean * 1e-6) / 1e9) if a else "-",
                 "%.3f" % (a / (mean * 1e-6) / 1e9 / 8000.0) if a else "-"]
        lines.append("| " + " | ".join(cells) + " |")
        if hbm:
            traffic[k] = {"fetch_kib": statistics.mean(fk[k]), "write_kib": statistics.mean(wk[k]),
                          "hbm_bytes_per_launch": hbm, "alg_bytes_per_launch": a, "mean_us": mean}
    return "\n".join(lines) + "\n", traffic


def _update_traffic(path, traffic):
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.dirname(here))
    from bench import csrc_hash
    data = {}
    if os.path.exists(path):
        data = json.load(open(path))
    if data.get("csrc_hash") != csrc_hash():
        data = {"csrc_hash": csrc_hash(), "kernels": {}}
    data["kernels"].update(traffic)
    json.dump(data, open(path, "w"), indent=1)


def main():
    ap = argparse.ArgumentParser()
    if len(sys.argv) > 1 and sys.argv[1] == "kernels":
        ap.add_argument("cmd")
        ap.add_argument("--trace", required=True)
        ap.add_argument("--fetch", required=True)
        ap.add_argument("--write", required=True)
        ap.add_argument("--copy-fetch", required=True)
        ap.add_argument("--copy-write", required=True)
        ap.add_argument("--alg", action="append", default=[],
                        help="kernel-name fragment=algorithmic bytes per dispatch (repeatable)")
        ap.add_argument("--title", required=True)
        ap.add_argument("--command", required=True)
        ap.add_argument("--counter-command", required=True)
        ap.add_argument("--note", default="")
        ap.add_argument("--out", required=True)
        ap.add_argument("--traffic-json", default="")
        a = ap.parse_args()
        alg = {}
        for item in a.alg:
            frag, v = item.rsplit("=", 1)
            alg[frag] = float(v)
        text, traffic = kernels_table(a.trace, a.fetch, a.write, a.copy_fetch, a.copy_write, alg, a.title, a.command,
                                      a.counter_command, a.note)
        with open(a.out, "w") as f:
            f.write(text)
        if a.traffic_json and traffic:
            _update_traffic(a.traffic_json, traffic)
        print(text)
        return
    if len(sys.argv) > 1 and sys.argv[1] == "stats":
        ap.add_argument("cmd")
        ap.add_argument("--trace", required=True)
        ap.add_argument("--title", required=True)
        ap.add_argument("--command", required=True)
        ap.add_argument("--note", default="")
        ap.add_argument("--out", required=True)
        a = ap.parse_args()
        text = stats_table(a.trace, a.title, a.command, a.note)
        with open(a.out, "w") as f:
            f.write(text)
        print(text)
        return
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--passes", required=True)
    ap.add_argument("--alg-bytes", type=float, required=True, help="algorithmic bytes per pass")
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--counter-command", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic-json", default="")
    a = ap.parse_args()
    names = a.passes.split(",")
    npass = len(names)

    trace = _fft_dispatches(_csv(a.trace, "kernel_trace.csv"))
    groups = _per_pass(trace, npass)
    lines = ["# " + a.title, "", "Command (kernel trace):", "", "    " + a.command, ""]
    lines += ["| pass | kernel | dispatches | mean us | min us | max us | alg GB/s (mean) |",
              "|---|---|---|---|---|---|---|"]
    summary = {}
    for name, g in zip(names, groups):
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in g]
        mean = statistics.mean(d)
        kern = g[0]["Kernel_Name"].split("(")[0]
        lines.append("| %s | `%s` | %d | %.1f | %.1f | %.1f | %.0f |" % (
            name, kern, len(d), mean, min(d), max(d), a.alg_bytes / (mean * 1e-6) / 1e9))
        summary[name] = {"kernel": kern, "mean_us": mean}
    lines.append("")
    traffic = {}
    if a.fetch and a.write and a.copy_fetch and a.copy_write:
        sf, sw, cf, cw = copy_scale(a.copy_fetch, a.copy_write)
        fr = _per_pass(_fft_dispatches(_csv(a.fetch, "counter_collection.csv")), npass)
        wr = _per_pass(_fft_dispatches(_csv(a.write, "counter_collection.csv")), npass)
        lines += ["Counters (separate runs, `--pmc FETCH_SIZE` then `--pmc WRITE_SIZE`):", "",
                  "    " + a.counter_command, "",
                  "Scale: a plain 1 GiB device copy reads FETCH_SIZE = %.1f KiB and "
                  "WRITE_SIZE = %.1f KiB, so FETCH_SIZE is multiplied by %.4f and WRITE_SIZE "
                  "by %.4f." % (cf, cw, sf, sw), "",
                  "| pass | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes / launch (scaled) | "
                  "/ algorithmic |", "|---|---|---|---|---|"]
        for name, f, w in zip(names, fr, wr):
            fk = statistics.mean(float(r["Counter_Value"]) for r in f)
            wk = statistics.mean(float(r["Counter_Value"]) for r in w)
            hbm = (fk * sf + wk * sw) * 1024.0
            traffic[name] = {"fetch_kib": fk, "write_kib": wk, "hbm_bytes_per_launch": hbm}
            lines.append("| %s | %.1f | %.1f | %.4g | %.4f |" % (name, fk, wk, hbm, hbm / a.alg_bytes))
        lines.append("")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if a.traffic_json and traffic:
        here = os.path.dirname(os.path.abspath(__file__))
        sys.path.insert(0, os.path.dirname(here))
        from bench import csrc_hash
        data = {}
        if os.path.exists(a.traffic_json):
            data = json.load(open(a.traffic_json))
        if data.get("csrc_hash") != csrc_hash():
            data = {"csrc_hash": csrc_hash(), "kernels": {}}
        data["kernels"].update(traffic)
        json.dump(data, open(a.traffic_json, "w"), indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
