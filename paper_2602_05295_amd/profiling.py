"""Summaries of rocprofv3 result databases (rocpd SQLite) for the profiles/
folder.

    python -m paper_2602_05295_amd.profiling trace  <results.db>  [--title T] [--command C]
    python -m paper_2602_05295_amd.profiling traffic <fetch.db> <write.db> --copy-bytes B
                                             --kernel NAME=FMT:BYTES_PER_LAUNCH [...] [--json OUT]
    python -m paper_2602_05295_amd.profiling valu <sq.db> --kernel NAME=FMT [...] --json OUT
    python -m paper_2602_05295_amd.profiling sq <sq.db> [<sq2.db> ...] --kernel NAME=LABEL:CELLS [...]

`trace` prints the per-kernel table of a --kernel-trace --stats run.
`traffic` turns two --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch,
summed over the counter's instances) into HBM bytes per launch.  Each counter
is scaled by the factor that makes it read the known size of a plain device
copy profiled in the same run (the largest __amd_rocclr_copyBuffer
dispatches): the copy moves B bytes each way.
`valu` records SQ_INSTS_VALU (wave instructions) per dispatch of the named
kernels, for the VALU-issue roofline bench.py reports beside the HBM one.
`sq` tabulates the SQ counters of one or more --pmc runs per named kernel
(means per dispatch): instruction mix, VALU per cell, waiting.
"""
from __future__ import annotations

import argparse
import json
import sqlite3
import sys
from collections import defaultdict


def kernel_table(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    con.close()
    return rows


def counter_per_dispatch(db: str):
    """{kernel name: [counter value per dispatch]} (instances summed)."""
    con = sqlite3.connect(db)
    acc = defaultdict(float)
    names = {}
    for disp, kn, v in con.execute("select dispatch_id, kernel_name, value from counters_collection"):
        acc[disp] += v
        names[disp] = kn
    con.close()
    out = defaultdict(list)
    for disp in sorted(acc):
        out[names[disp]].append(acc[disp])
    return out


def counter_per_dispatch_named(db: str, counter: str):
    """{kernel name: [value of `counter` per dispatch]} (instances summed)."""
    con = sqlite3.connect(db)
    acc = defaultdict(float)
    names = {}
    for disp, kn, v in con.execute(
            "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?", (counter,)):
        acc[disp] += v
        names[disp] = kn
    con.close()
    out = defaultdict(list)
    for disp in sorted(acc):
        out[names[disp]].append(acc[disp])
    return out


def copy_scale(per: dict, copy_bytes: int) -> float:
    vals = [v for v in per.get("__amd_rocclr_copyBuffer", []) if v * 1024 > copy_bytes / 8]
    if not vals:
        raise SystemExit("no calibration copy found in the counter database")
    return copy_bytes / (sum(vals) / len(vals) * 1024)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    q = sub.add_parser("valu")
    q.add_argument("db", help="a --pmc run holding SQ_INSTS_VALU")
    q.add_argument("--kernel", action="append", default=[], help="NAME=FMT")
    q.add_argument("--json", required=True)
    q.add_argument("--kernel-hash", default=None)
    c = sub.add_parser("sq")
    c.add_argument("db", nargs="+", help="--pmc runs holding SQ_ / GRBM_ counters")
    c.add_argument("--kernel", action="append", default=[], help="NAME=LABEL:CELLS_PER_LAUNCH")
    r = sub.add_parser("traffic")
    r.add_argument("fetch_db")
    r.add_argument("write_db")
    r.add_argument("--copy-bytes", type=int, required=True)
    r.add_argument("--kernel", action="append", default=[], help="NAME=FMT:ALGORITHMIC_BYTES_PER_LAUNCH")
    r.add_argument("--json", default=None)
    r.add_argument("--kernel-hash", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "valu":
        per = counter_per_dispatch_named(a.db, "SQ_INSTS_VALU")
        res = {"kernel_hash": a.kernel_hash, "counter": "SQ_INSTS_VALU (wave instructions per dispatch)",
               "formats": {}}
        for spec in a.kernel:
            name, fmt = spec.rsplit("=", 1)
            vals = per.get(name)
            if not vals:
                print(f"missing kernel {name}", file=sys.stderr)
                return 1
            res["formats"][fmt] = {"kernel": name, "dispatches": len(vals),
                                   "valu_instructions_per_launch": round(sum(vals) / len(vals))}
            print(fmt, res["formats"][fmt])
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)
            fh.write("\n")
        return 0
    if a.cmd == "sq":
        # mean per dispatch of every counter found, then the derived columns
        means = defaultdict(dict)
        for db in a.db:
            con = sqlite3.connect(db)
            names = {row[0] for row in con.execute("select distinct counter_name from counters_collection")}
            con.close()
            for cn in sorted(names):
                for kn, vals in counter_per_dispatch_named(db, cn).items():
                    means[kn][cn] = sum(vals) / len(vals)
        print("| kernel | waves | VALU instr | VALU / cell | LDS instr | VMEM rd instr | wait | VALU active | "
              "LDS bank conflicts |")
        print("|---|---:|---:|---:|---:|---:|---:|---:|---:|")
        for spec in a.kernel:
            name, rest = spec.rsplit("=", 1)
            label, cells = rest.rsplit(":", 1)
            m = means.get(name)
            if not m:
                print(f"missing kernel {name}", file=sys.stderr)
                return 1
            g = lambda k: m.get(k, float("nan"))
            wc = g("SQ_WAVE_CYCLES")
            print(f"| `{name}` ({label}) | {g('SQ_WAVES'):.0f} | {g('SQ_INSTS_VALU') / 1e6:.1f} M | "
                  f"{g('SQ_INSTS_VALU') * 64 / int(cells):.0f} | {g('SQ_INSTS_LDS') / 1e6:.1f} M | "
                  f"{g('SQ_INSTS_VMEM_RD') / 1e6:.2f} M | {g('SQ_WAIT_INST_ANY') / wc:.2f} | "
                  f"{g('SQ_ACTIVE_INST_VALU') / wc:.2f} | {g('SQ_LDS_BANK_CONFLICT'):.0f} |")
        return 0
    if a.cmd == "trace":
        print("| kernel | calls | total (us) | average (us) | share |")
        print("|---|---:|---:|---:|---:|")
        for name, calls, tot, avg, pct in kernel_table(a.db):
            print(f"| `{name}` | {calls} | {tot:.1f} | {avg:.2f} | {pct:.2f}% |")
        return 0
    F = counter_per_dispatch(a.fetch_db)
    W = counter_per_dispatch(a.write_db)
    fs, ws = copy_scale(F, a.copy_bytes), copy_scale(W, a.copy_bytes)
    res = {"kernel_hash": a.kernel_hash, "copy_bytes": a.copy_bytes, "fetch_scale": round(fs, 5),
           "write_scale": round(ws, 5), "formats": {}}
    print(f"scale factors: FETCH_SIZE x{fs:.4f}, WRITE_SIZE x{ws:.4f} (a {a.copy_bytes}-byte copy)")
    print("| kernel | dispatches | fetch (B) | write (B) | total (B) | algorithmic (B) | ratio |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for spec in a.kernel:
        name, rest = spec.rsplit("=", 1)
        fmt, alg = rest.split(":")
        alg = int(alg)
        fv, wv = F.get(name), W.get(name)
        if not fv or not wv:
            print(f"missing kernel {name}", file=sys.stderr)
            return 1
        f = sum(fv) / len(fv) * 1024 * fs
        w = sum(wv) / len(wv) * 1024 * ws
        res["formats"][fmt] = {"kernel": name, "dispatches": len(fv), "fetch_bytes": round(f), "write_bytes": round(w),
                               "hbm_bytes_per_launch": round(f + w), "algorithmic_bytes": alg,
                               "ratio": round((f + w) / alg, 4)}
        print(f"| `{name}` | {len(fv)} | {f:.4g} | {w:.4g} | {f + w:.4g} | {alg} | {(f + w) / alg:.3f} |")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)
            fh.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
