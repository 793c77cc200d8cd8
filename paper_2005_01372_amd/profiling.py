"""Summaries of rocprofv3 output for the committed profile records.

``kernel_stats``: turns a ``--kernel-trace --stats --output-format csv`` run
into a short text table.  ``traffic``: turns two ``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE`` runs (of a command that also performs one plain device
copy of known size and dumps the library's event profile) into HBM bytes per
launch for one kernel function, each counter scaled by what it reads for the
copy.  Usage::

    python -m paper_2005_01372_amd.profiling stats <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_2005_01372_amd.profiling traffic <fetch.csv> <write.csv> <copy_bytes> <kernel function> \
        <profile dump.json> <out.json> "<command>"
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_sha():
    """Hash of every source file of the library (kernels, launch settings, host plans): a change to any of them
    marks counter records taken before it as stale."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(HERE, "..", "include", "lsop.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name, width=70):
    name = name.replace("void ", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def kernel_stats(csv_path, out_path, command, top=15):
    rows = list(csv.DictReader(open(csv_path)))
    key_name = "Name" if "Name" in rows[0] else "KernelName"
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"rocprofv3 kernel-trace statistics", f"command: {command}", "",
             f"{'kernel':70s} {'calls':>6s} {'total ms':>10s} {'avg ms':>9s} {'%':>6s}"]
    for r in rows[:top]:
        lines.append(f"{_short(r[key_name]):70s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e6:9.4f} {float(r['Percentage']):6.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return lines


def _dispatches(csv_path, counter):
    """[(dispatch id, kernel name, bytes)] for one counter (KiB per dispatch -> bytes), in dispatch order."""
    out = []
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
    out.sort()
    return out


def _copy_scale(disp, copy_bytes):
    """copy_bytes over what the counter read for the first plain copy of at least 1 MiB (the probe, issued
    before anything else; later copies, such as a bandwidth measurement, are of other sizes)."""
    for _, name, v in disp:
        if "lsop::" in name:
            break
        if "copyBuffer" in name and v >= (1 << 20):
            return copy_bytes / v
    raise SystemExit("no copy probe found before the first library kernel")


def traffic(fetch_csv, write_csv, copy_bytes, kernel_fns, dump_json, out_path, command):
    """HBM bytes per launch of each kernel function (``;``-separated names) over its algorithmic bytes.

    The counter runs are of bench.py with --copy-probe (a plain 1 GiB copy
    first, which scales each counter to bytes) and --dump-profile (the
    library's own event profile of the timed region: launches and
    algorithmic bytes per kernel function).  The timed region is the end of
    the run, so its launches are the last `launches` dispatches of the kernel.
    """
    dumps = json.load(open(dump_json))["kernels"]
    disp = {c: _dispatches(p, c) for c, p in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv))}
    scale = {c: _copy_scale(d, copy_bytes) for c, d in disp.items()}
    kernels = {}
    for kernel_fn in [k for k in kernel_fns.split(";") if k]:
        dump = dumps[kernel_fn]
        nl = int(dump["launches"])
        tot = {}
        for counter, d in disp.items():
            mine = [v for _, name, v in d if (kernel_fn + "(") in name][-nl:]
            if len(mine) != nl:
                raise SystemExit(f"{counter}: found {len(mine)} dispatches of {kernel_fn}, expected {nl}")
            tot[counter] = scale[counter] * sum(mine)
        kernels[kernel_fn] = {
            "dispatches": nl,
            "fetch_bytes_per_launch": tot["FETCH_SIZE"] / nl, "write_bytes_per_launch": tot["WRITE_SIZE"] / nl,
            "algorithmic_bytes_per_launch": dump["bytes"] / nl,
            "hbm_over_algorithmic": (tot["FETCH_SIZE"] + tot["WRITE_SIZE"]) / dump["bytes"]}
    rec = {"source_sha": kernel_source_sha(), "command": command, "copy_bytes": copy_bytes,
           "copy_scale": scale, "kernels": kernels}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print("\n".join(kernel_stats(sys.argv[2], sys.argv[3], sys.argv[4])))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6],
                                 sys.argv[7], sys.argv[8]), indent=1))
