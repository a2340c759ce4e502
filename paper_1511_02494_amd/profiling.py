"""rocprofv3 summaries for the selected-SpMV bench.

Turns the CSV output of three rocprofv3 runs of ``bench.py`` (one
``--kernel-trace --stats`` run, one ``--pmc FETCH_SIZE`` run, one
``--pmc WRITE_SIZE`` run) into the short text summaries kept in ``profiles/``
and the per-kernel traffic record ``bench.py`` reads for its roofline.

HBM bytes are calibrated in the same runs: the bench's bandwidth probe reads
a buffer of known size with ``k_read`` and copies it with ``k_copy``, so
bytes = counter * (known bytes / counter of the probe kernel).

    python -m paper_1511_02494_amd.profiling --stats DIR --fetch DIR --write DIR \\
        --cmd-stats "..." --cmd-fetch "..." --cmd-write "..." --workload "..." \\
        --stats-md profiles/A.md --traffic-md profiles/B.md --traffic-json profiles/C.json
    python -m paper_1511_02494_amd.profiling counters --dirs D1 D2 --cmds "..." "..." \\
        --kernels PREFIX... --title "..." --out profiles/D.md
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE_BYTES = 4 << 30  # buffer size bench.py hands to spmv_hbm_probe


def kernel_source_hash() -> str:
    """SHA-256 of the HIP sources, to tell whether stored counters still apply."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1511_02494_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode() + f.read())
    return h.hexdigest()


def stored_traffic(path: str, kernel_prefixes, cold: bool = True) -> float | None:
    """HBM bytes per launch (fetch + write, summed over the given kernels)
    from a traffic record, or None when it is missing, was taken on other
    kernel sources, or lacks one of the kernels.  ``cold``: the dispatches
    that ran right after a cache flush (the bench's cold launches), when the
    record has them."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    total = 0.0
    for name in kernel_prefixes:
        hits = [v for k, v in rec["kernels"].items() if k.startswith(name)]
        if not hits:
            return None
        h = hits[0]
        if cold and h.get("cold_dispatches"):
            total += h["cold_fetch_bytes"] + h["cold_write_bytes"]
        else:
            total += h["fetch_bytes"] + h["write_bytes"]
    return total


def _one(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def read_stats(d: str):
    rows = []
    with open(_one(d, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append(dict(name=r["Name"], calls=int(r["Calls"]),
                             total_ms=float(r["TotalDurationNs"]) / 1e6,
                             avg_us=float(r["AverageNs"]) / 1e3, min_us=float(r["MinNs"]) / 1e3,
                             max_us=float(r["MaxNs"]) / 1e3, pct=float(r["Percentage"])))
    return sorted(rows, key=lambda r: -r["total_ms"])


def read_counter(d: str, counter: str):
    """kernel name -> list of per-dispatch values (KiB) of one counter."""
    out = defaultdict(list)
    with open(_one(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


FLUSH = "spmvsel::k_flush"


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise SystemExit(f"none of {names} in the CSV columns {sorted(row)}")


def cold_flags(names):
    """For a dispatch sequence (in issue order), True for the dispatches of
    the execute that follows each cache flush: the bench's cold leg flushes,
    runs one execute (one to three kernels, none twice) and waits, so the
    group is the dispatches after a flush up to three of them, ending early
    at another flush or at a kernel already in the group (the next execute)."""
    out = [False] * len(names)
    i = 0
    while i < len(names):
        if names[i].startswith(FLUSH):
            seen = set()
            j = i + 1
            while j < len(names) and j <= i + 3 and not names[j].startswith(FLUSH) \
                    and names[j] not in seen:
                seen.add(names[j])
                out[j] = True
                j += 1
            i = j
        else:
            i += 1
    return out


def read_trace(d: str):
    """Kernel dispatches of a --kernel-trace run in issue order: (name, ns)."""
    rows = []
    with open(_one(d, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((int(_col(r, "Dispatch_Id", "Correlation_Id")), r["Kernel_Name"],
                         int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))))
    rows.sort()
    return [(n, t) for _, n, t in rows]


def read_counter_dispatches(d: str, counter: str):
    """Per dispatch of a --pmc run, in issue order: (name, value KiB); the
    flush dispatches included (value None if the counter row is missing)."""
    by = {}
    with open(_one(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            k = int(_col(r, "Dispatch_Id", "Correlation_Id"))
            if k not in by:
                by[k] = [r["Kernel_Name"], None]
            if r["Counter_Name"] == counter:
                by[k][1] = (by[k][1] or 0.0) + float(r["Counter_Value"])
    return [tuple(by[k]) for k in sorted(by)]


def cold_warm_means(seq):
    """name -> dict(cold_mean, cold_n, warm_mean, warm_n) over (name, value) pairs."""
    flags = cold_flags([n for n, _ in seq])
    acc = defaultdict(lambda: [0.0, 0, 0.0, 0])
    for (n, v), c in zip(seq, flags):
        if v is None:
            continue
        a = acc[n]
        if c:
            a[0] += v
            a[1] += 1
        else:
            a[2] += v
            a[3] += 1
    return {n: dict(cold_mean=a[0] / a[1] if a[1] else None, cold_n=a[1],
                    warm_mean=a[2] / a[3] if a[3] else None, warm_n=a[3]) for n, a in acc.items()}


def _short(name: str, n: int = 100) -> str:
    return name if len(name) <= n else name[:n] + "..."


def _find(d, prefix):
    for k, v in d.items():
        if k.startswith(prefix):
            return v
    raise SystemExit(f"calibration kernel {prefix} not in the counter run")


# Derived shares of the busy time, from counters rocprofv3 sums over the
# device: GRBM_GUI_ACTIVE over the 8 XCDs, the TA/TCP counters over the 256
# CUs.  (name, numerator, denominator kind)
XCDS, CUS = 8, 256
DERIVED = [
    ("address unit busy", "TA_TA_BUSY_sum", "cu"),
    ("address unit stalled by L1", "TA_ADDR_STALLED_BY_TC_CYCLES_sum", "cu"),
    ("L1 waiting on L2", "TCP_PENDING_STALL_CYCLES_sum", "cu"),
    ("L1 tag conflicts", "TCP_READ_TAGCONFLICT_STALL_CYCLES_sum", "cu"),
]


def derived_columns(m):
    """Derived metrics of one kernel's counter means m (missing -> None)."""
    out = {}
    cyc = m.get("GRBM_GUI_ACTIVE")
    if cyc:
        cyc /= XCDS
        out["busy us (2.4 GHz)"] = cyc / 2.4e3
        for name, num, _ in DERIVED:
            if num in m:
                out[name] = m[num] / (CUS * cyc)
    if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m and m["TCC_HIT_sum"] + m["TCC_MISS_sum"] > 0:
        out["L2 hit rate"] = m["TCC_HIT_sum"] / (m["TCC_HIT_sum"] + m["TCC_MISS_sum"])
    if m.get("TCP_TCC_READ_REQ_sum"):
        if "TCP_TCC_READ_REQ_LATENCY_sum" in m:
            out["L2 read latency (cycles)"] = m["TCP_TCC_READ_REQ_LATENCY_sum"] / m["TCP_TCC_READ_REQ_sum"]
        if "TCP_TOTAL_CACHE_ACCESSES_sum" in m:
            out["L1 accesses per L2 read"] = m["TCP_TOTAL_CACHE_ACCESSES_sum"] / m["TCP_TCC_READ_REQ_sum"]
    return out


def counters_main(argv):
    """Per-kernel means of arbitrary counters from several --pmc runs of the
    same command; --by-grid keeps launches of different grid sizes (different
    matrices) apart, and the derived shares follow where their counters are
    present."""
    ap = argparse.ArgumentParser(prog="profiling counters")
    ap.add_argument("--dirs", nargs="+", required=True)
    ap.add_argument("--cmds", nargs="+", required=True)
    ap.add_argument("--kernels", nargs="+", required=True, help="kernel name prefixes to report")
    ap.add_argument("--title", required=True)
    ap.add_argument("--notes", default="")
    ap.add_argument("--by-grid", action="store_true")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    vals = defaultdict(lambda: defaultdict(list))
    order = []
    for d in a.dirs:
        with open(_one(d, "counter_collection.csv")) as f:
            per = defaultdict(dict)  # one dispatch: counter -> summed value
            for r in csv.DictReader(f):
                if not any(r["Kernel_Name"].startswith(k) for k in a.kernels):
                    continue
                c = r["Counter_Name"]
                if c not in order:
                    order.append(c)
                key = (r["Kernel_Name"], r.get("Grid_Size", "") if a.by_grid else "")
                disp = per[(key, r["Dispatch_Id"])]
                disp[c] = disp.get(c, 0.0) + float(r["Counter_Value"])
            for (key, _), cs in per.items():
                for c, v in cs.items():
                    vals[key][c].append(v)
    rows = []
    for key in sorted(vals):
        m = {c: sum(v) / len(v) for c, v in vals[key].items() if v}
        rows.append((key, m, derived_columns(m)))
    dnames = []
    for _, _, dv in rows:
        for k in dv:
            if k not in dnames:
                dnames.append(k)
    with open(a.out, "w") as f:
        f.write(f"# {a.title}\n\nCommands (repository root, one MI355X), one counter group per "
                "run:\n\n" + "".join(f"    {c}\n" for c in a.cmds) + "\n")
        if a.notes:
            f.write(a.notes + "\n\n")
        label = "kernel | grid" if a.by_grid else "kernel"
        if dnames:
            f.write("Derived (busy time = GRBM_GUI_ACTIVE / 8 XCDs; shares of it per CU):\n\n")
            f.write(f"| {label} | " + " | ".join(dnames) + " |\n|---|" + ("---|" if a.by_grid else "")
                    + "---:|" * len(dnames) + "\n")
            for (name, grid), m, dv in rows:
                cells = " | ".join(f"{dv[k]:.3g}" if k in dv else "" for k in dnames)
                g = f" | {grid}" if a.by_grid else ""
                f.write(f"| `{_short(name, 60)}`{g} | {cells} |\n")
            f.write("\n")
        f.write("Mean per dispatch (rocprofv3 sums each counter over the device).\n\n")
        f.write(f"| {label} | " + " | ".join(order) + " |\n|---|" + ("---|" if a.by_grid else "")
                + "---:|" * len(order) + "\n")
        for (name, grid), m, _ in rows:
            g = f" | {grid}" if a.by_grid else ""
            f.write(f"| `{_short(name, 60)}`{g} | " + " | ".join(f"{m.get(c, float('nan')):.4g}" for c in order) + " |\n")
    print(f"wrote {a.out}")


def stats_main(argv):
    """Kernel-time table of one --kernel-trace --stats run, limited to the
    kernels whose names start with one of --kernels (all if none given)."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--kernels", nargs="*", default=[])
    ap.add_argument("--notes", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    rows = [r for r in read_stats(a.dir)
            if not a.kernels or any(r["name"].startswith(k) for k in a.kernels)]
    with open(a.out, "w") as f:
        f.write(f"# {a.title}\n\nWorkload: {a.workload}\n\nCommand (repository root, one "
                f"MI355X):\n\n    {a.cmd}\n\n")
        if a.notes:
            f.write(a.notes + "\n\n")
        f.write("| kernel | calls | total ms | average us | min us | max us | % of all |\n"
                "|---|---:|---:|---:|---:|---:|---:|\n")
        for r in rows:
            f.write(f"| `{_short(r['name'])}` | {r['calls']} | {r['total_ms']:.2f} | "
                    f"{r['avg_us']:.1f} | {r['min_us']:.1f} | {r['max_us']:.1f} | "
                    f"{r['pct']:.2f} |\n")
    print(f"wrote {a.out}")


def main(argv=None):
    import sys
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "counters":
        return counters_main(argv[1:])
    if argv and argv[0] == "stats":
        return stats_main(argv[1:])
    ap = argparse.ArgumentParser()
    for k in ("stats", "fetch", "write", "cmd-stats", "cmd-fetch", "cmd-write", "workload",
              "stats-md", "traffic-md", "traffic-json"):
        ap.add_argument("--" + k, required=True)
    a = ap.parse_args(argv)

    stats = read_stats(a.stats)
    cw = cold_warm_means(read_trace(a.stats))
    with open(a.stats_md, "w") as f:
        f.write("# Kernel time summary: selected-SpMV bench\n\n")
        f.write(f"Workload: {a.workload}\n\nCommand (repository root, one MI355X):\n\n"
                f"    {a.cmd_stats}\n\n")
        f.write("## SpMV kernels, cold and warm dispatches\n\nCold: the dispatches of an execute "
                "that follows a cache flush (the bench's roofline leg); warm: all others (the "
                "timed solver loops).  Means of the kernel trace's durations.\n\n"
                "| kernel | cold dispatches | cold mean us | warm dispatches | warm mean us |\n"
                "|---|---:|---:|---:|---:|\n")
        for n in sorted(cw, key=lambda k: -(cw[k]["cold_mean"] or 0)):
            c = cw[n]
            if not c["cold_n"] or not n.startswith("void spmvsel::k_"):
                continue
            f.write(f"| `{_short(n)}` | {c['cold_n']} | {c['cold_mean'] / 1e3:.1f} | {c['warm_n']} | "
                    f"{(c['warm_mean'] or 0) / 1e3:.1f} |\n")
        f.write("\n## All kernels (rocprofv3 --stats)\n\n")
        f.write("| kernel | calls | total ms | average us | min us | max us | % |\n"
                "|---|---:|---:|---:|---:|---:|---:|\n")
        for r in stats:
            f.write(f"| `{_short(r['name'])}` | {r['calls']} | {r['total_ms']:.2f} | "
                    f"{r['avg_us']:.1f} | {r['min_us']:.1f} | {r['max_us']:.1f} | "
                    f"{r['pct']:.2f} |\n")

    fetch = read_counter(a.fetch, "FETCH_SIZE")
    write = read_counter(a.write, "WRITE_SIZE")
    rd = _find(fetch, "spmvsel::k_read")
    cp = _find(write, "spmvsel::k_copy")
    kib = PROBE_BYTES / 1024
    fscale = kib / (sum(rd) / len(rd))
    wscale = kib / (sum(cp) / len(cp))
    fcw = cold_warm_means(read_counter_dispatches(a.fetch, "FETCH_SIZE"))
    wcw = cold_warm_means(read_counter_dispatches(a.write, "WRITE_SIZE"))
    kernels = {}
    for name in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(name, []), write.get(name, [])
        fk = sum(fv) / len(fv) if fv else 0.0
        wk = sum(wv) / len(wv) if wv else 0.0
        kernels[name] = dict(dispatches=max(len(fv), len(wv)), fetch_kib=fk, write_kib=wk,
                             fetch_bytes=fk * 1024 * fscale, write_bytes=wk * 1024 * wscale)
        fc, wc = fcw.get(name, {}), wcw.get(name, {})
        if fc.get("cold_n") and wc.get("cold_n"):
            kernels[name].update(cold_dispatches=fc["cold_n"],
                                 cold_fetch_bytes=fc["cold_mean"] * 1024 * fscale,
                                 cold_write_bytes=wc["cold_mean"] * 1024 * wscale)
    rec = dict(source_sha256=kernel_source_hash(), fetch_scale=fscale, write_scale=wscale,
               probe_bytes=PROBE_BYTES, commands=[a.cmd_fetch, a.cmd_write], kernels=kernels)
    with open(a.traffic_json, "w") as f:
        json.dump(rec, f, indent=1)
    with open(a.traffic_md, "w") as f:
        f.write("# HBM traffic per dispatch (rocprofv3 PMC): selected-SpMV bench\n\n")
        f.write(f"Workload: {a.workload}\n\nCommands (repository root, one MI355X), one counter "
                f"per run:\n\n    {a.cmd_fetch}\n    {a.cmd_write}\n\n")
        f.write(f"Calibration in the same runs (bandwidth probe, {PROBE_BYTES >> 30} GiB buffer): "
                f"`k_read` FETCH_SIZE scale {fscale:.3f}, `k_copy` WRITE_SIZE scale "
                f"{wscale:.3f} (true bytes per counter byte). Mean per dispatch.\n\n")
        f.write("Cold: dispatches of an execute right after a cache flush (the bench's roofline "
                "leg).\n\n| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled fetch MB | "
                "scaled write MB | cold dispatches | cold fetch MB | cold write MB |\n"
                "|---|---:|---:|---:|---:|---:|---:|---:|---:|\n")
        for name, v in kernels.items():
            cold = (f"{v['cold_dispatches']} | {v['cold_fetch_bytes'] / 1e6:.1f} | "
                    f"{v['cold_write_bytes'] / 1e6:.1f}") if v.get("cold_dispatches") else "0 | | "
            f.write(f"| `{_short(name)}` | {v['dispatches']} | {v['fetch_kib']:.0f} | "
                    f"{v['write_kib']:.0f} | {v['fetch_bytes'] / 1e6:.1f} | "
                    f"{v['write_bytes'] / 1e6:.1f} | {cold} |\n")
    print(f"wrote {a.stats_md}, {a.traffic_md}, {a.traffic_json}")


if __name__ == "__main__":
    main()
