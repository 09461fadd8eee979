"""Summaries of rocprofv3 result databases (host-only tool).

  python -m paper_2605_16684_amd.rocprof_report stats DB --cmd "..." [--out FILE]
      kernel table (calls, average and total duration) from a
      `rocprofv3 --kernel-trace --stats` run;
  python -m paper_2605_16684_amd.rocprof_report traffic FETCH_DB WRITE_DB
          --workload NAME --cmd-fetch "..." --cmd-write "..." [--out FILE] [--json FILE]
      HBM bytes per launch of each stage kernel from `--pmc FETCH_SIZE` and
      `--pmc WRITE_SIZE` runs, each scaled by what the same counter reads for
      the library's copy kernel of known size (1 GiB read + 1 GiB written,
      run by `bench.py --calib-copy`);
  python -m paper_2605_16684_amd.rocprof_report flops PMC_DB TRACE_DB
          --workload NAME --cmd-pmc "..." --cmd-trace "..." [--out FILE]
      executed FP64 work of each stage kernel from a `--pmc` run of the
      SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 and SQ_INSTS_VALU_FLOPS_FP64
      counters, divided by the kernel's average duration in a kernel trace,
      against the MI355X FP64 vector peak.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sqlite3
import sys

COPY_BYTES = 1 << 30


def _rows(db, sql, args=()):
    con = sqlite3.connect(db)
    try:
        return list(con.execute(sql, args))
    finally:
        con.close()


def kernel_stats(db):
    return _rows(db, "select name, total_calls, total_duration, average from top_kernels "
                     "order by total_duration desc")


def counter_by_kernel(db, counter):
    out = collections.defaultdict(list)
    for name, val in _rows(db, "select kernel_name, value from counters_collection "
                               "where counter_name = ? order by dispatch_id", (counter,)):
        out[name].append(val)
    return out


def _copy_factor(per_kernel):
    vals = [v for k, vs in per_kernel.items() if "copy_kernel" in k for v in vs]
    if not vals:
        raise SystemExit("no esdg::copy_kernel dispatch in the counter run (use --calib-copy)")
    kib = sum(vals) / len(vals)
    return COPY_BYTES / (kib * 1024.0), kib


def cmd_stats(a):
    rows = kernel_stats(a.db)
    lines = [f"# rocprofv3 kernel trace: {a.title}", "", "Command:", "", "```", a.cmd, "```", "",
             "| kernel | calls | avg (us) | total (us) |", "|---|---:|---:|---:|"]
    for name, calls, total, avg in rows:
        lines.append(f"| `{name[:110]}` | {calls} | {avg:.2f} | {total:.1f} |")
    txt = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt)


def cmd_traffic(a):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2605_16684_amd import perfmodel
    fetch = counter_by_kernel(a.fetch_db, "FETCH_SIZE")
    write = counter_by_kernel(a.write_db, "WRITE_SIZE")
    ff, fkib = _copy_factor(fetch)
    wf, wkib = _copy_factor(write)
    lines = [f"# HBM traffic per launch: {a.workload}", "",
             "Commands (FETCH_SIZE pass, then WRITE_SIZE pass):", "", "```", a.cmd_fetch,
             a.cmd_write, "```", "",
             f"Calibration with the library copy kernel (1 GiB read + 1 GiB written): "
             f"FETCH_SIZE reads {fkib:.0f} KiB -> factor {ff:.4f}; "
             f"WRITE_SIZE reads {wkib:.0f} KiB -> factor {wf:.4f}.", "",
             "| kernel | launches | FETCH (MB, scaled) | WRITE (MB, scaled) | total (MB) |",
             "|---|---:|---:|---:|---:|"]
    rec = {}
    for name in sorted(fetch):
        if "stage_" not in name or name not in write:
            continue
        fv, wv = fetch[name], write[name]
        n = min(len(fv), len(wv))
        fb = sum(fv[:n]) / n * 1024.0 * ff
        wb = sum(wv[:n]) / n * 1024.0 * wf
        lines.append(f"| `{name}` | {n} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} |")
        mode = "rhs" if name.rstrip(")").split("(")[0].rstrip(">").endswith(" 0") else "stage"
        rec[name] = {"mode": mode, "fetch_bytes": fb, "write_bytes": wb,
                     "bytes_per_launch": fb + wb}
    txt = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt)
    if a.json:
        data = {}
        if os.path.exists(a.json):
            with open(a.json) as f:
                data = json.load(f)
        for name, r in rec.items():
            # the curved kernels of a run are recorded under the warped mesh's workload
            ent = data.setdefault(a.workload + ("_curved" if "stage_curved" in name else ""), {})
            key = "stage_fp64" if (r["mode"] == "stage" and "stage_fp64" in name) else name
            r = dict(r, kernel=name,
                     kernel_hash=perfmodel.kernel_source_hash(
                         names=perfmodel.kernel_sources(name)),
                     fetch_factor=ff, write_factor=wf)
            ent[key] = r
        with open(a.json, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


F64_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU_FLOPS_FP64",
                "SQ_INSTS_VALU_FLOPS_FP64_TRANS", "SQ_INSTS_VALU", "SQ_WAVES")


def cmd_flops(a):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2605_16684_amd import perfmodel
    per = {c: counter_by_kernel(a.pmc_db, c) for c in F64_COUNTERS}
    durations = {name: avg for name, calls, total, avg in kernel_stats(a.trace_db)}
    lines = [f"# Executed FP64 work per launch: {a.workload}", "",
             "Commands (counter pass, then kernel trace for the durations):", "", "```",
             a.cmd_pmc, a.cmd_trace, "```", "",
             "Executed FP64 FLOPs = 64 lanes x (ADD + MUL + TRANS + 2 FMA) wave instructions "
             "(an upper bound: the last wave of a 125-lane workgroup has 61 active lanes); "
             "the FLOPS_FP64 x 64 column is the hardware's FLOP counter (which counts per wave "
             "instruction) times the lanes, as a cross-check. Peak: "
             f"{perfmodel.FP64_VECTOR_TFLOPS} TF/s FP64 vector.", "",
             "| kernel | launches | VALU instr./wave | FP64 add/mul/fma/trans (M wave-instr.) "
             "| FLOPs (instr., G) | FLOPS_FP64 x 64 (G) | avg (us) | executed TF/s | of peak |",
             "|---|---:|---:|---|---:|---:|---:|---:|---:|"]
    for name in sorted(per["SQ_INSTS_VALU_FMA_F64"]):
        if "stage_" not in name:
            continue
        avg = {c: (sum(v) / len(v) if v else float("nan"))
               for c, v in ((c, per[c].get(name, [])) for c in F64_COUNTERS)}
        n = len(per["SQ_INSTS_VALU_FMA_F64"][name])
        fl = 64.0 * (avg["SQ_INSTS_VALU_ADD_F64"] + avg["SQ_INSTS_VALU_MUL_F64"]
                     + avg["SQ_INSTS_VALU_TRANS_F64"] + 2.0 * avg["SQ_INSTS_VALU_FMA_F64"])
        hw = 64.0 * (avg["SQ_INSTS_VALU_FLOPS_FP64"] + avg["SQ_INSTS_VALU_FLOPS_FP64_TRANS"])
        dur = durations.get(name)
        tf = fl / (dur * 1e-6) / 1e12 if dur else float("nan")
        lines.append(
            f"| `{name[:70]}` | {n} | {avg['SQ_INSTS_VALU'] / avg['SQ_WAVES']:.0f} | "
            f"{avg['SQ_INSTS_VALU_ADD_F64'] / 1e6:.1f} / {avg['SQ_INSTS_VALU_MUL_F64'] / 1e6:.1f} / "
            f"{avg['SQ_INSTS_VALU_FMA_F64'] / 1e6:.1f} / {avg['SQ_INSTS_VALU_TRANS_F64'] / 1e6:.2f} | "
            f"{fl / 1e9:.2f} | {hw / 1e9:.2f} | {dur if dur else float('nan'):.1f} | {tf:.1f} | "
            f"{tf / perfmodel.FP64_VECTOR_TFLOPS:.2f} |")
    txt = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt)


def cmd_mix(a):
    """Instruction mix per wave of the stage kernels, from one or more
    counter passes of the same command (each pass counts SQ_WAVES too)."""
    per = {}
    for db in a.dbs:
        waves = counter_by_kernel(db, "SQ_WAVES")
        for row in _rows(db, "select distinct counter_name from counters_collection"):
            c = row[0]
            if c == "SQ_WAVES":
                continue
            for name, vals in counter_by_kernel(db, c).items():
                if "stage_" not in name or name not in waves:
                    continue
                w = sum(waves[name]) / len(waves[name])
                per.setdefault(name, {})[c] = sum(vals) / len(vals) / w
    counters = sorted({c for r in per.values() for c in r})
    names = sorted(per)
    lines = [f"# Instruction mix per wave: {a.workload}", "", "Commands (one counter pass each):",
             "", "```", *a.cmd, "```", "",
             "Average count per wave over the launches of each kernel (SQ counters divided by "
             "SQ_WAVES of the same pass).", "",
             "| counter | " + " | ".join(f"`{n[:48]}`" for n in names) + " |",
             "|---|" + "---:|" * len(names)]
    for c in counters:
        lines.append(f"| {c} | " + " | ".join(
            f"{per[n][c]:.0f}" if c in per[n] else "" for n in names) + " |")
    txt = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--out")
    s.set_defaults(fn=cmd_stats)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--workload", required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out")
    t.add_argument("--json")
    t.set_defaults(fn=cmd_traffic)
    f = sub.add_parser("flops")
    f.add_argument("pmc_db")
    f.add_argument("trace_db")
    f.add_argument("--workload", required=True)
    f.add_argument("--cmd-pmc", required=True)
    f.add_argument("--cmd-trace", required=True)
    f.add_argument("--out")
    f.set_defaults(fn=cmd_flops)
    m = sub.add_parser("mix")
    m.add_argument("dbs", nargs="+")
    m.add_argument("--workload", required=True)
    m.add_argument("--cmd", action="append", required=True)
    m.add_argument("--out")
    m.set_defaults(fn=cmd_mix)
    a = ap.parse_args(argv)
    a.fn(a)


if __name__ == "__main__":
    main()
