"""Summaries of rocprofv3 CSV output for the committed profiles.

  python -m paper_1107_5415_amd.profsum stats STATS_CSV --cmd "..." --out FILE
      [--trace TRACE_CSV --tail-kernel NAME --tail-n N [--tail-kernel ... --tail-n ...]]
      per-kernel calls / total / average duration from --kernel-trace --stats,
      and the average of the last N dispatches of each named kernel
  python -m paper_1107_5415_amd.profsum sq CSV [CSV ...] --write-csv WRITE_CSV --copy-kib KIB
      --cmd "..." [--cmd "..."] --out FILE
      per-kernel averages per dispatch of the SQ counters in the CSVs, with
      VALU lane-operations per complex point (SQ_INSTS_VALU * 64 / points,
      points = output bytes / 8 from the calibrated WRITE_SIZE run) and the
      ratio of wait to VALU instructions
  python -m paper_1107_5415_amd.profsum traffic FETCH_CSV WRITE_CSV --kernel NAME
      --copy-kib KIB --alg-bytes B --sources F1,F2 --cmd-fetch "..." --cmd-write "..."
      --out JSON [--alg-per-write R]
      HBM bytes per launch of NAME from FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch), each scaled by what the same counter reads for the plain
      copy kernel of COPY-KIB KiB in the same run.
"""
import argparse
import csv
import hashlib
import json
import os
import statistics
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_KERNEL = "copyBuffer"


def _short(name):
    return name.replace("lfft::(anonymous namespace)::", "").replace(
        "(lfft::PassDesc, HIP_vector_type<float, 2u> const*, HIP_vector_type<float, 2u>*)", "")


def stats(path, cmd, out, trace=None, tails=()):
    rows = list(csv.DictReader(open(path)))
    lines = ["# rocprofv3 --kernel-trace --stats summary", "# command: " + cmd, "",
             "%-72s %7s %12s %11s %6s" % ("kernel", "calls", "total_us", "avg_us", "pct")]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append("%-72s %7d %12.1f %11.2f %6.2f" % (
            _short(r["Name"])[:72], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    if trace and tails:
        # the last tail_n dispatches of each kernel (the benchmark's traced
        # pass runs last), from the per-dispatch kernel trace
        rows_tr = list(csv.DictReader(open(trace)))
        lines.append("")
        for tail_kernel, tail_n in tails:
            tr = [r for r in rows_tr if tail_kernel in r["Kernel_Name"]]
            tr.sort(key=lambda r: int(r["Start_Timestamp"]))
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr[-tail_n:]]
            lines.append("# last %d dispatches of %s (the traced pass): avg_us %.2f, min %.2f, max %.2f"
                         % (len(d), tail_kernel, statistics.mean(d), min(d), max(d)))
    open(out, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    per = {}
    for (name, _), v in sorted(vals.items(), key=lambda kv: int(kv[0][1])):
        per.setdefault(name, []).append(v)
    return per


def digest(sources):
    h = hashlib.sha256()
    for s in sources:
        with open(os.path.join(CSRC, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic(fetch_csv, write_csv, kernel, copy_kib, alg_bytes, sources, cmd_f, cmd_w, out,
            alg_per_write=None):
    fe = _per_dispatch(fetch_csv, "FETCH_SIZE")
    wr = _per_dispatch(write_csv, "WRITE_SIZE")

    def bare(name):
        # "void ns::kernel<args>(params)" -> "kernel<args>"
        n = name.replace("lfft::(anonymous namespace)::", "").replace("lfft::", "")
        if n.startswith("void "):
            n = n[5:]
        depth = 0
        for i, ch in enumerate(n):
            if ch == "<":
                depth += 1
            elif ch == ">":
                depth -= 1
            elif ch == "(" and depth == 0:
                return n[:i].strip()
        return n.strip()

    def find(d, key, exact=True):
        hits = [k for k in d if (bare(k) == key if exact else key in k)]
        if len(hits) != 1:
            raise SystemExit("kernel %r matched %d names" % (key, len(hits)))
        return d[hits[0]]
    # the calibration copy is the largest device copy of the run (the other
    # copies are small host-to-device uploads of inputs and masks)
    cf = max(find(fe, COPY_KERNEL, exact=False))
    cw = max(find(wr, COPY_KERNEL, exact=False))
    sf = copy_kib / cf
    sw = copy_kib / cw
    f_all = [x * sf * 1024 for x in find(fe, kernel)]
    w_all = [x * sw * 1024 for x in find(wr, kernel)]
    extra = {}
    if alg_per_write is None:
        # mean over the kernel's dispatches (the run's launch mix must be the
        # benchmark's)
        kf = statistics.mean(f_all)
        kw = statistics.mean(w_all)
    else:
        # launches of several sizes: the two runs dispatch the same sequence,
        # so dispatch i pairs across them; its algorithmic bytes are
        # alg_per_write times its (exact, write-once) output bytes.  The
        # measured / algorithmic ratio over every dispatch scales the
        # benchmark's per-launch algorithmic bytes.
        if len(f_all) != len(w_all):
            raise SystemExit("dispatch counts differ: %d vs %d" % (len(f_all), len(w_all)))
        alg = [alg_per_write * w for w in w_all]
        rf = sum(f_all) / sum(alg)
        rw = sum(w_all) / sum(alg)
        kf = rf * alg_bytes
        kw = rw * alg_bytes
        extra = {"dispatches": len(f_all), "alg_per_write": alg_per_write,
                 "traffic_over_alg": rf + rw}
    data = json.load(open(out)) if os.path.exists(out) else {}
    data[kernel] = {
        "bytes_per_launch": kf + kw,
        "fetch_bytes_per_launch": kf,
        "write_bytes_per_launch": kw,
        "alg_bytes_per_launch": alg_bytes,
        **extra,
        "copy_scale": {"fetch": sf, "write": sw, "copy_kib": copy_kib},
        "sources": sources,
        "source_digest": digest(sources),
        "commands": [cmd_f, cmd_w],
    }
    json.dump(data, open(out, "w"), indent=1)
    print(json.dumps(data[kernel]))


def sq(csvs, write_csv, copy_kib, cmds, out):
    vals = {}
    for path in csvs:
        per = {}
        for r in csv.DictReader(open(path)):
            key = (_short(r["Kernel_Name"]), r["Counter_Name"])
            per.setdefault(key, {}).setdefault(r["Dispatch_Id"], 0.0)
            per[key][r["Dispatch_Id"]] += float(r["Counter_Value"])
        for (k, c), d in per.items():
            vals.setdefault(k, {})[c] = statistics.mean(d.values())
    wr = _per_dispatch(write_csv, "WRITE_SIZE")
    cw = max(v for k, l in wr.items() if COPY_KERNEL in k for v in l)
    scale = copy_kib / cw
    points = {}
    for k, l in wr.items():
        points[_short(k)] = statistics.mean(l) * scale * 1024 / 8
    cols = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "SQ_INSTS_SALU",
            "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"]
    lines = ["# rocprofv3 --pmc SQ counters, averages per dispatch over the run (all launches of each kernel)"]
    lines += ["# command: " + c for c in cmds]
    lines += ["# lane_ops_per_point = SQ_INSTS_VALU * 64 / points; points = WRITE_SIZE bytes / 8 per dispatch "
              "(calibrated on the run's largest device copy); wait/valu = SQ_WAIT_INST_ANY / SQ_INSTS_VALU", ""]
    lines.append("%-56s" % "kernel" + "".join("%16s" % c.replace("SQ_", "") for c in cols) +
                 "%12s%10s" % ("ops/point", "wait/valu"))
    order = sorted(vals, key=lambda k: -vals[k].get("SQ_WAVE_CYCLES", 0))
    for k in order:
        v = vals[k]
        pts = points.get(k)
        ops = v.get("SQ_INSTS_VALU", 0) * 64 / pts if pts else float("nan")
        wv = v.get("SQ_WAIT_INST_ANY", 0) / v["SQ_INSTS_VALU"] if v.get("SQ_INSTS_VALU") else float("nan")
        lines.append("%-56s" % k[:56] + "".join("%16.1f" % v.get(c, float("nan")) for c in cols) +
                     "%12.1f%10.2f" % (ops, wv))
    open(out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what")
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--trace", default=None)
    s.add_argument("--tail-kernel", action="append", default=[])
    s.add_argument("--tail-n", type=int, action="append", default=[])
    q = sub.add_parser("sq")
    q.add_argument("csvs", nargs="+")
    q.add_argument("--write-csv", required=True)
    q.add_argument("--copy-kib", type=float, required=True)
    q.add_argument("--cmd", action="append", required=True)
    q.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-kib", type=float, required=True)
    t.add_argument("--alg-bytes", type=float, required=True)
    t.add_argument("--sources", required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--alg-per-write", type=float, default=None)
    a = ap.parse_args()
    if a.what == "stats":
        if len(a.tail_kernel) != len(a.tail_n):
            raise SystemExit("--tail-kernel and --tail-n come in pairs")
        stats(a.csv, a.cmd, a.out, a.trace, list(zip(a.tail_kernel, a.tail_n)))
    elif a.what == "sq":
        sq(a.csvs, a.write_csv, a.copy_kib, a.cmd, a.out)
    elif a.what == "traffic":
        traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_kib, a.alg_bytes, a.sources.split(","),
                a.cmd_fetch, a.cmd_write, a.out, a.alg_per_write)
    else:
        ap.print_help()
        sys.exit(2)


if __name__ == "__main__":
    main()
