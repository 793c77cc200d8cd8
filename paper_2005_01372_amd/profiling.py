"""Summaries of rocprofv3 output for the committed profile records.

``kernel_stats``: turns a ``--kernel-trace --stats --output-format csv`` run
into a short text table.  ``traffic``: turns two ``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE`` runs (of a command that also performs one plain device
copy of known size) into HBM bytes per launch for one kernel, each counter
scaled by what it reads for the copy.  Usage::

    python -m paper_2005_01372_amd.profiling stats <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_2005_01372_amd.profiling traffic <fetch.csv> <write.csv> <copy_bytes> <kernel substring> \
        <lib name> <out.json> "<command>" <nx,lx,lz,element bytes>
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("kernels_fft.hip", "kernels_la.hip", "fft_engine.hpp"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
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


def cols_algorithmic_bytes(name, grid_size, nx, lx, lz, esize):
    """Algorithmic bytes of one column-pass dispatch, from its template tile width and grid size."""
    c = int(name.split("<")[1].split(">")[0].split(",")[2])
    g = 64 if lx >= 512 else {32: 8, 64: 8, 96: 8, 128: 16, 192: 8, 256: 32, 384: 16, 768: 32}[lx]
    pz = 2 * lz
    wgs = grid_size // (c * g)
    nslots = wgs // (pz // c)
    return nslots * 2.0 * nx * pz * esize + 2.0 * pz * lx * esize


def _per_dispatch(csv_path, counter, geom=None):
    """{kernel name: [(bytes, algorithmic bytes) per dispatch]} plus the copy dispatches issued before the first
    library kernel."""
    out, copies, seen_lib = {}, [], False
    rows = sorted(csv.DictReader(open(csv_path)), key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"]) * 1024.0  # KiB -> bytes
        name = r["Kernel_Name"]
        seen_lib = seen_lib or "lsop::" in name
        if "copyBuffer" in name and not seen_lib and v >= (1 << 20):
            copies.append(v)
        alg = cols_algorithmic_bytes(name, int(r["Grid_Size"]), *geom) if (geom and "k_cols<" in name) else None
        out.setdefault(name, []).append((v, alg))
    return out, copies


def traffic(fetch_csv, write_csv, copy_bytes, kernel_substr, lib_name, out_path, command, geom):
    fetch, fcopy = _per_dispatch(fetch_csv, "FETCH_SIZE", geom)
    write, wcopy = _per_dispatch(write_csv, "WRITE_SIZE", geom)
    sf, sw = copy_bytes / sum(fcopy), copy_bytes / sum(wcopy)
    names = [k for k in fetch if kernel_substr in k]
    if not names:
        raise SystemExit(f"no kernel matching {kernel_substr!r}")
    f = [v for k in names for v in fetch[k]]
    w = [v for k in names for v in write.get(k, [])]
    fb, wb = sf * sum(v for v, _ in f), sw * sum(v for v, _ in w)
    alg = sum(a for _, a in f)
    rec = {
        "source_sha": kernel_source_sha(), "command": command, "copy_bytes": copy_bytes,
        "copy_scale": {"FETCH_SIZE": sf, "WRITE_SIZE": sw},
        "kernels": {lib_name: {
            "rocprof_names": names, "dispatches": len(f),
            "fetch_bytes_per_launch": fb / len(f), "write_bytes_per_launch": wb / len(w),
            "algorithmic_bytes_per_launch": alg / len(f),
            "hbm_over_algorithmic": (fb + wb) / alg}},
    }
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print("\n".join(kernel_stats(sys.argv[2], sys.argv[3], sys.argv[4])))
    elif sys.argv[1] == "traffic":
        geom = tuple(int(v) for v in sys.argv[9].split(","))  # nx, lx, lz, bytes per complex element
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6],
                                 sys.argv[7], sys.argv[8], geom), indent=1))
