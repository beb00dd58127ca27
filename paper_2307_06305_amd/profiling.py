"""Memory-traffic measurement from rocprofv3 counters.

Two counter runs of `bench.py --profile` (one with FETCH_SIZE, one with
WRITE_SIZE, both in KiB per dispatch) give the HBM bytes of the SpMV kernels.
Each counter is scaled by what it reads for the copy probe of known size
(`damn_stream_copy`), launched in the same run:

    bytes = counter_KiB * 1024 / (copy_counter_KiB * 1024 / copy_bytes)

    python -m paper_2307_06305_amd.profiling summarize \\
        --fetch <fetch run>/run_counter_collection.csv \\
        --write <write run>/run_counter_collection.csv \\
        --copy-bytes 1073741824 --out profiles/spmv_27pt128_traffic.md

The summary records a hash of the kernel sources; bench.py reports the
traffic only while the sources still hash the same.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
# the product kernels and the host code that cuts their tiles
KERNEL_SOURCES = ("csrc/spmv_kernels.hip", "csrc/spmv_templates.h", "csrc/damn_device.h",
                  "csrc/api.hip")
DA_LAUNCH = "stream_g2_t1024"   # launch shapes the counter runs use by default
CSR_LAUNCH = "stream_g2_t1024"


def stream_launch(name):
    """(lanes, tile, gather) of a stream launch name: stream_gG_tT for
    interleaved gathers (gather 1), paired_gG_tT for paired ones (2)."""
    m = re.fullmatch(r"(stream|paired)_g(\d+)_t(\d+)", name)
    if not m:
        raise ValueError(f"not a stream launch name: {name!r}")
    return int(m.group(2)), int(m.group(3)), 2 if m.group(1) == "paired" else 1


def kernel_name(label, launch):
    g, _, x = stream_launch(launch)
    index = "short" if label == "da" else "int"
    # the last two template arguments are the matrix stream's cache policy
    # (2: non-temporal) and the x values per gather load
    return (f"spmv_stream<{index}, double, {'true' if label == 'da' else 'false'}, {g}, false, "
            f"double, 2, {x}>")
COPY_KERNEL = "stream_copy"


def _code_only(text):
    """C++ source without comments and with whitespace collapsed, so that
    editing a comment does not invalidate a recorded measurement."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def _per_kernel(path, counter):
    """Mean counter value per dispatch, by kernel name."""
    sums, counts = {}, {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            name = row["Kernel_Name"]
            sums[name] = sums.get(name, 0.0) + float(row["Counter_Value"])
            counts[name] = counts.get(name, 0) + 1
    return {k: (sums[k] / counts[k], counts[k]) for k in sums}


def _find(table, needle):
    for name, v in table.items():
        if needle in name:
            return v
    raise KeyError(f"no kernel matching {needle!r}")


def summarize(fetch_csv, write_csv, copy_bytes, launch_da=DA_LAUNCH, launch_csr=CSR_LAUNCH):
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    cf = _find(fetch, COPY_KERNEL)[0] * 1024 / copy_bytes
    cw = _find(write, COPY_KERNEL)[0] * 1024 / copy_bytes
    out = {"copy_bytes": copy_bytes, "fetch_scale": cf, "write_scale": cw,
           "source_sha256": kernel_source_hash(), "kernels": {}}
    for label, launch in (("da", launch_da), ("csr", launch_csr)):
        needle = kernel_name(label, launch)
        fk, nf = _find(fetch, needle)
        wk, nw = _find(write, needle)
        out["kernels"][label] = {
            "kernel": needle, "launch": launch, "dispatches": [nf, nw], "fetch_kib": fk,
            "write_kib": wk,
            "hbm_read_bytes": fk * 1024 / cf, "hbm_write_bytes": wk * 1024 / cw,
            "hbm_bytes": fk * 1024 / cf + wk * 1024 / cw}
    return out


TITLE_27PT = "DA-CSR and CSR SpMV, 3D 27-point stencil 128^3"
MODEL_27PT = "Traffic model (Eq. 3 plus x once and y written): DA 599,372,724 B, CSR 710,858,660 B."


def write_summary(summary, path, command, title=TITLE_27PT, model=MODEL_27PT):
    da, csr = summary["kernels"]["da"], summary["kernels"]["csr"]
    lines = [
        f"# HBM traffic: {title}",
        "",
        "Counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch), one rocprofv3 run each:",
        "",
        "```",
        command,
        "```",
        "",
        f"Copy probe ({summary['copy_bytes']} bytes read and written): FETCH_SIZE reads "
        f"{summary['fetch_scale']:.4f} and WRITE_SIZE {summary['write_scale']:.4f} of the "
        "known bytes; the kernels' counters are divided by these factors.",
        "",
        "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read B | HBM write B | total B |",
        "|---|---:|---:|---:|---:|---:|",
    ]
    for k in (da, csr):
        lines.append(f"| `{k['kernel']}` ({k['launch']}) | {k['fetch_kib']:.0f} | {k['write_kib']:.0f} | "
                     f"{k['hbm_read_bytes']:.4g} | {k['hbm_write_bytes']:.4g} | "
                     f"{k['hbm_bytes']:.4g} |")
    lines += ["", model, "", "```json", json.dumps(summary, indent=1), "```", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def read_traffic(path, label="da", launch=None):
    """HBM bytes per launch recorded in a summary, or None if the summary is
    missing, the kernel sources changed since it was taken, or it recorded
    another launch shape than `launch`."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    s = json.loads(m.group(1))
    if s.get("source_sha256") != kernel_source_hash():
        return None
    k = s["kernels"][label]
    if launch is not None and k.get("launch") != launch:
        return None
    return k["hbm_bytes"]


def kernel_stats(stats_csv, needles=None):
    """(name, calls, avg us, min us, max us, share %) from a rocprofv3
    --stats kernel table, largest total time first; needles (substrings)
    keep only the kernels that match one of them."""
    rows = []
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            name = r["Name"].replace("void ", "").split("(")[0]
            if needles and not any(n in name for n in needles):
                continue
            rows.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                         float(r["Percentage"]), float(r["TotalDurationNs"])))
    rows.sort(key=lambda t: -t[6])
    return [t[:6] for t in rows]


def write_trace_summary(stats_csv, path, title, command, notes, needles=None, top=24):
    lines = [f"# {title}", "", "Command (run from the repository root on one MI355X; `cd /tmp` "
             "first):", "", "```", command, "```", ""]
    lines += [notes, "", "| kernel | calls | avg us | min us | max us | share % |",
              "|---|---:|---:|---:|---:|---:|"]
    for name, calls, avg, mn, mx, pct in kernel_stats(stats_csv, needles)[:top]:
        lines.append(f"| `{name}` | {calls} | {avg:.1f} | {mn:.1f} | {mx:.1f} | {pct:.2f} |")
    lines.append("")
    with open(path, "w") as f:
        f.write("\n".join(lines))


def counter_means(csv_paths):
    """{kernel name: {counter: mean value per dispatch}} over rocprofv3
    counter-collection CSVs (one per --pmc pass)."""
    sums, counts = {}, {}
    for path in csv_paths:
        with open(path) as f:
            for row in csv.DictReader(f):
                name = row["Kernel_Name"].replace("void ", "").split("(")[0]
                key = (name, row["Counter_Name"])
                sums[key] = sums.get(key, 0.0) + float(row["Counter_Value"])
                counts[key] = counts.get(key, 0) + 1
    out = {}
    for (name, counter), v in sums.items():
        out.setdefault(name, {})[counter] = v / counts[(name, counter)]
    return out


def dispatch_groups(trace_csv, needles):
    """(name, threads in the grid, dispatches, avg us, min us) from a rocprofv3
    kernel-trace CSV, grouped by kernel and grid size (launches of one
    kernel with different grids, such as the read probe's one-pass and
    many-pass launches, kept apart)."""
    groups = {}
    with open(trace_csv) as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"].replace("void ", "").split("(")[0]
            if not any(k in name for k in needles):
                continue
            us = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
            groups.setdefault((name, int(row["Grid_Size_X"])), []).append(us)
    return [(n, g, len(v), sum(v) / len(v), min(v)) for (n, g), v in sorted(groups.items())]


def write_group_summary(traces, path, title, command, notes, needles):
    """Per trace (label=path), the kernel-and-grid groups of dispatch_groups."""
    lines = [f"# {title}", "", "Commands (run from the repository root on one MI355X; `cd /tmp` "
             "first):", "", "```", command, "```", "", notes, ""]
    for spec in traces:
        label, trace = spec.split("=", 1)
        lines += [f"## {label}", "", "| kernel | grid threads | dispatches | avg us | min us |",
                  "|---|---:|---:|---:|---:|"]
        for n, g, k, avg, mn in dispatch_groups(trace, needles):
            lines.append(f"| `{n}` | {g} | {k} | {avg:.1f} | {mn:.1f} |")
        lines.append("")
    with open(path, "w") as f:
        f.write("\n".join(lines))


def write_counter_summary(specs, path, title, command, notes, needles):
    """A table of counters (rows) by workload and kernel (columns), means per
    dispatch, for the kernels that match `needles`.  specs: label=csv[,csv...]
    (one CSV per counter set of one workload)."""
    cols = []  # (label, kernel, {counter: mean})
    for spec in specs:
        label, paths = spec.split("=", 1)
        means = counter_means(paths.split(","))
        for name in means:
            if any(k in name for k in needles):
                cols.append((label, name, means[name]))
    counters = sorted({c for _, _, m in cols for c in m})
    lines = [f"# {title}", "", "Commands (run from the repository root on one MI355X; `cd /tmp` "
             "first), one rocprofv3 run per counter set:", "", "```", command, "```", "",
             notes, ""]
    lines.append("| counter | " + " | ".join(f"{lb}: `{n}`" for lb, n, _ in cols) + " |")
    lines.append("|---|" + "---:|" * len(cols))
    for c in counters:
        lines.append(f"| {c} | " + " | ".join(
            f"{m[c]:.6g}" if c in m else "" for _, _, m in cols) + " |")
    lines.append("")
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2307_06305_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("trace", help="summarise a rocprofv3 --stats kernel table")
    tr.add_argument("--stats", required=True)
    tr.add_argument("--out", required=True)
    tr.add_argument("--title", required=True)
    tr.add_argument("--command", required=True)
    tr.add_argument("--notes", default="")
    tr.add_argument("--match", nargs="*", default=None)
    tr.add_argument("--top", type=int, default=24)
    gr = sub.add_parser("groups", help="kernel-trace durations by kernel and grid size")
    gr.add_argument("--trace", nargs="+", required=True, help="label=run_kernel_trace.csv")
    gr.add_argument("--out", required=True)
    gr.add_argument("--title", required=True)
    gr.add_argument("--command", required=True)
    gr.add_argument("--notes", default="")
    gr.add_argument("--match", nargs="+", required=True)
    cn = sub.add_parser("counters", help="table of counter means per dispatch by kernel")
    cn.add_argument("--csv", nargs="+", required=True,
                    help="label=csv[,csv...]: one workload's counter-collection CSVs")
    cn.add_argument("--out", required=True)
    cn.add_argument("--title", required=True)
    cn.add_argument("--command", required=True)
    cn.add_argument("--notes", default="")
    cn.add_argument("--match", nargs="+", required=True)
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--copy-bytes", type=int, required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="")
    s.add_argument("--launch-da", default=DA_LAUNCH)
    s.add_argument("--launch-csr", default=CSR_LAUNCH)
    s.add_argument("--title", default=TITLE_27PT)
    s.add_argument("--model", default=MODEL_27PT)
    a = ap.parse_args(argv)
    if a.cmd == "groups":
        write_group_summary(a.trace, a.out, a.title, a.command, a.notes, a.match)
        return 0
    if a.cmd == "counters":
        write_counter_summary(a.csv, a.out, a.title, a.command, a.notes, a.match)
        return 0
    if a.cmd == "trace":
        write_trace_summary(a.stats, a.out, a.title, a.command, a.notes, a.match, a.top)
        return 0
    summary = summarize(a.fetch, a.write, a.copy_bytes, a.launch_da, a.launch_csr)
    write_summary(summary, a.out, a.command, a.title, a.model)
    print(json.dumps(summary["kernels"]), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
