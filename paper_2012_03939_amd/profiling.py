"""rocprofv3 helpers: the plain-copy reference for the HBM byte counters and the
summaries kept under profiles/.

    python -m paper_2012_03939_amd.profiling copyref
        a plain 512 MiB device-to-device copy (three times), the reference that
        scales FETCH_SIZE / WRITE_SIZE to bytes
    python -m paper_2012_03939_amd.profiling pmc --fetch D1 --write D2 --copy-fetch D3 --copy-write D4
                                            [--sq D5 ...] --out FILE.json --command "..."
        per-kernel counter summary (KiB per dispatch, copy-scaled HBM bytes per dispatch)
    python -m paper_2012_03939_amd.profiling trace --stats run_kernel_stats.csv --out FILE.md --title "..."
                                              --command "..."
        kernel-time table of a --kernel-trace --stats run

Counter summaries carry the hash of the HIP sources they were taken on; bench.py
reports the measured traffic only while that hash matches.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 512 << 20          # bytes read and written by one copy of the reference


def kernel_source_hash() -> str:
    """Hash of the HIP sources (csrc/*): counter summaries are valid only for these."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def copy_reference(reps: int = 3):
    import torch
    a = torch.ones(COPY_BYTES // 4, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {COPY_BYTES} bytes x{reps}", flush=True)


def _short(name: str) -> str:
    n = name.split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return n[4:] if n.startswith("st::") else n


def read_counters(d: str):
    """{kernel: {counter: [value per dispatch]}} and {kernel: [duration ns per dispatch]}."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    vals = collections.defaultdict(lambda: collections.defaultdict(dict))
    dur = collections.defaultdict(dict)
    for fn in files:
        with open(fn) as fh:
            for row in csv.DictReader(fh):
                k = _short(row["Kernel_Name"])
                disp = row["Dispatch_Id"]
                c = row["Counter_Name"]
                vals[k][c][disp] = vals[k][c].get(disp, 0.0) + float(row["Counter_Value"])
                dur[k][disp] = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
    out = {k: {c: list(v.values()) for c, v in cs.items()} for k, cs in vals.items()}
    return out, {k: list(v.values()) for k, v in dur.items()}


def _copy_factor(d: str, counter: str) -> float:
    vals, _ = read_counters(d)
    per = [v for k, cs in vals.items() if "copyBuffer" in k or "copy" in k.lower() for v in cs.get(counter, [])]
    if not per:
        raise ValueError(f"no copy dispatch with {counter} in {d}")
    kib = max(per)              # the 512 MiB copy is the largest copy dispatch
    return COPY_BYTES / (kib * 1024.0)


def pmc_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, sq_dirs=(), command="") -> dict:
    ff = _copy_factor(copy_fetch_dir, "FETCH_SIZE")
    wf = _copy_factor(copy_write_dir, "WRITE_SIZE")
    fv, fdur = read_counters(fetch_dir)
    wv, _ = read_counters(write_dir)
    sv = collections.defaultdict(dict)
    for d in sq_dirs or ():
        for k, cs in read_counters(d)[0].items():
            sv[k].update(cs)
    kernels = {}
    for k in sorted(fv):
        f = fv[k].get("FETCH_SIZE")
        w = wv.get(k, {}).get("WRITE_SIZE")
        if not f or not w:
            continue
        n = len(f)
        e = {"dispatches": n,
             "fetch_kib_per_dispatch": sum(f) / n,
             "write_kib_per_dispatch": sum(w) / len(w),
             "mean_dispatch_ms_under_counters": sum(fdur[k]) / len(fdur[k]) / 1e6}
        e["hbm_bytes_per_dispatch"] = (e["fetch_kib_per_dispatch"] * ff + e["write_kib_per_dispatch"] * wf) * 1024.0
        for c in ("TCC_HIT_sum", "TCC_MISS_sum"):
            if c in wv.get(k, {}):
                e[c.lower() + "_per_dispatch"] = sum(wv[k][c]) / len(wv[k][c])
        if "tcc_hit_sum_per_dispatch" in e and "tcc_miss_sum_per_dispatch" in e:
            t = e["tcc_hit_sum_per_dispatch"] + e["tcc_miss_sum_per_dispatch"]
            e["l2_hit_rate"] = e["tcc_hit_sum_per_dispatch"] / t if t else None
        for c, v in sv.get(k, {}).items():
            e[c.lower() + "_per_dispatch"] = sum(v) / len(v)
        if e.get("sq_thread_cycles_valu_per_dispatch") and e.get("sq_active_inst_valu_per_dispatch"):
            # active lanes per VALU instruction cycle, over the 64 of a wave
            e["valu_lane_utilisation"] = (e["sq_thread_cycles_valu_per_dispatch"]
                                          / e["sq_active_inst_valu_per_dispatch"] / 64.0)
        kernels[k] = e
    return {"command": command, "source_hash": kernel_source_hash(), "fetch_size_factor": ff,
            "write_size_factor": wf, "copy_reference_bytes": COPY_BYTES, "kernels": kernels}


def trace_table(stats_csv: str, top: int = 24):
    rows = []
    with open(stats_csv) as fh:
        for r in csv.DictReader(fh):
            rows.append((_short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                         float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda r: -r[2])
    lines = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows[:top]:
        lines.append(f"| {name} | {calls} | {tot:.2f} | {avg:.1f} | {pct:.2f} |")
    return "\n".join(lines)


def busy_phases(trace_csv: str, gap_ms: float = 100.0):
    """Split a rocprofv3 kernel trace at idle gaps longer than gap_ms and report,
    per phase, the wall time from its first kernel start to its last kernel end,
    the time during which at least one kernel ran (union of the intervals), the
    summed kernel durations, the launch count and the kernels by summed time."""
    ev = []
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"])))
    ev.sort()
    phases, cur, last_end = [], [], None
    for e in ev:
        if cur and e[0] - last_end > gap_ms * 1e6:
            phases.append(cur)
            cur = []
        cur.append(e)
        last_end = e[1] if last_end is None or not cur[:-1] else max(last_end, e[1])
    if cur:
        phases.append(cur)
    out = []
    for ph in phases:
        busy, s0, e0 = 0, None, None
        for a, b, _ in ph:
            if e0 is None or a > e0:
                if e0 is not None:
                    busy += e0 - s0
                s0, e0 = a, b
            else:
                e0 = max(e0, b)
        busy += e0 - s0
        per = collections.defaultdict(float)
        for a, b, n in ph:
            per[n] += (b - a) / 1e6
        out.append({"wall_ms": (max(b for _, b, _ in ph) - ph[0][0]) / 1e6, "busy_ms": busy / 1e6,
                    "kernel_sum_ms": sum((b - a) for a, b, _ in ph) / 1e6, "launches": len(ph),
                    "kernels": dict(sorted(per.items(), key=lambda kv: -kv[1]))})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copyref")
    p = sub.add_parser("pmc")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--out"):
        p.add_argument(a, required=True)
    p.add_argument("--sq", action="append", default=[], help="counter directory of an SQ pass (repeatable)")
    p.add_argument("--command", default="")
    t = sub.add_parser("trace")
    t.add_argument("--stats", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--title", default="Kernel times")
    t.add_argument("--command", default="")
    t.add_argument("--notes", default="")
    b = sub.add_parser("busy")
    b.add_argument("--trace", required=True, help="run_kernel_trace.csv of a --kernel-trace run")
    b.add_argument("--gap-ms", type=float, default=100.0)
    a = ap.parse_args(argv)
    if a.cmd == "busy":
        print(json.dumps(busy_phases(a.trace, a.gap_ms), indent=1))
        return 0
    if a.cmd == "copyref":
        copy_reference()
    elif a.cmd == "pmc":
        s = pmc_summary(a.fetch, a.write, a.copy_fetch, a.copy_write, a.sq, a.command)
        with open(a.out, "w") as fh:
            json.dump(s, fh, indent=1)
        print(f"wrote {a.out}: {', '.join(s['kernels'])}")
    else:
        body = [f"# {a.title}", ""]
        if a.notes:
            body += [a.notes, ""]
        body += ["Command (run from the repository root):", "", "```", a.command, "```", "",
                 trace_table(a.stats), ""]
        with open(a.out, "w") as fh:
            fh.write("\n".join(body))
        print(f"wrote {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
