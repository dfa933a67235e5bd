"""Summaries of rocprofv3 CSV output for the committed profiles.

  python -m paper_1107_5415_amd.profsum stats STATS_CSV --cmd "..." --out FILE
      per-kernel calls / total / average duration from --kernel-trace --stats
  python -m paper_1107_5415_amd.profsum traffic FETCH_CSV WRITE_CSV --kernel NAME
      --copy-kib KIB --alg-bytes B --sources F1,F2 --cmd-fetch "..." --cmd-write "..."
      --out JSON
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


def stats(path, cmd, out):
    rows = list(csv.DictReader(open(path)))
    lines = ["# rocprofv3 --kernel-trace --stats summary", "# command: " + cmd, "",
             "%-72s %7s %12s %11s %6s" % ("kernel", "calls", "total_us", "avg_us", "pct")]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append("%-72s %7d %12.1f %11.2f %6.2f" % (
            _short(r["Name"])[:72], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    open(out, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    per = {}
    for (name, _), v in vals.items():
        per.setdefault(name, []).append(v)
    return per


def digest(sources):
    h = hashlib.sha256()
    for s in sources:
        with open(os.path.join(CSRC, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic(fetch_csv, write_csv, kernel, copy_kib, alg_bytes, sources, cmd_f, cmd_w, out):
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
    # mean over the kernel's dispatches: the same launch mix as the
    # benchmark's per-launch average
    kf = statistics.mean(find(fe, kernel)) * sf * 1024
    kw = statistics.mean(find(wr, kernel)) * sw * 1024
    data = json.load(open(out)) if os.path.exists(out) else {}
    data[kernel] = {
        "bytes_per_launch": kf + kw,
        "fetch_bytes_per_launch": kf,
        "write_bytes_per_launch": kw,
        "alg_bytes_per_launch": alg_bytes,
        "copy_scale": {"fetch": sf, "write": sw, "copy_kib": copy_kib},
        "sources": sources,
        "source_digest": digest(sources),
        "commands": [cmd_f, cmd_w],
    }
    json.dump(data, open(out, "w"), indent=1)
    print(json.dumps(data[kernel]))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what")
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--out", required=True)
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
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.csv, a.cmd, a.out)
    elif a.what == "traffic":
        traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_kib, a.alg_bytes, a.sources.split(","),
                a.cmd_fetch, a.cmd_write, a.out)
    else:
        ap.print_help()
        sys.exit(2)


if __name__ == "__main__":
    main()
