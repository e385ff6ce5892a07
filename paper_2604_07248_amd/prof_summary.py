"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_2604_07248_amd.prof_summary stats DIR
        Markdown table of a `--kernel-trace --stats --output-format csv` run.
    python -m paper_2604_07248_amd.prof_summary pmc DIR [DIR ...]
        Per-kernel average of every counter of `--pmc ... --output-format csv` runs.
    python -m paper_2604_07248_amd.prof_summary traffic --fetch DIR --write DIR
            --copy-fetch DIR --copy-write DIR --copy-bytes B --leg NAME
        HBM bytes per launch of each kernel family: FETCH_SIZE and WRITE_SIZE
        (KiB per dispatch) scaled by what the same counters read for the
        library's copy kernel moving B bytes each way.  Ends with a JSON block
        that bench.py reads; it carries a hash of the library sources, so that
        figures taken on other kernels are not reported for these.

Kernel families are the ones turpy_profile uses.
"""

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def sources_sha256():
    """Hash of every kernel and schedule source of the library (csrc/)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if p.endswith((".hip", ".hpp", ".h")):
            h.update(os.path.basename(p).encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def family(kernel_name):
    """turpy_profile family of a kernel, from its demangled name."""
    n = kernel_name
    if "turpy::" not in n:
        return None  # runtime and PyTorch kernels
    m = re.search(r"row_(?:pair|pass)_kernel<(\d+), (\d+), (true|false)>", n)
    if m:
        if m.group(2) == "0":
            return "row_plain"
        return "row_bwd" if m.group(3) == "true" else "row_fwd"
    for key, fam in (("col_pair_kernel", "col_synth"), ("col_pass_kernel", "col"), ("synth_col_kernel", "synth"),
                     ("sh_kernel", "sh"), ("evolve_kernel", "evolve"), ("stats_kernel", "stats"),
                     ("finalize_kernel", "finalize"), ("copy_kernel", "copy"), ("recv_row_in", "recv_row"),
                     ("recv_col_grad", "recv_col_grad"), ("recv_col", "recv_col"),
                     ("recv_row_grad", "recv_row_grad"), ("recv_reduce", "recv_reduce")):
        if key in n:
            return fam
    return None


def short(kernel_name):
    n = re.sub(r"turpy::\(anonymous namespace\)::", "", kernel_name)
    n = re.sub(r"^void ", "", n)
    n = re.sub(r"\(turpy::\w+(, turpy::\w+)?(, long)?\)", "", n)
    return n[:70]


def _csv(dirname, suffix):
    files = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {dirname}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def stats_table(dirname):
    rows = _csv(dirname, "kernel_stats.csv")
    out = ["| kernel | family | calls | total us | average us | % |", "|---|---|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| {short(r['Name'])} | {family(r['Name']) or '-'} | {r['Calls']} | "
                   f"{float(r['TotalDurationNs']) / 1e3:.0f} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f} |")
    return out


def pmc_by_kernel(dirname):
    """{kernel name: {counter: average value per dispatch}}."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for r in _csv(dirname, "counter_collection.csv"):
        per[(r["Kernel_Name"], r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for (name, _), counters in per.items():
        for c, v in counters.items():
            acc[name][c].append(v)
    return {k: {c: (sum(v) / len(v), len(v)) for c, v in cs.items()} for k, cs in acc.items()}


def pmc_table(dirs):
    out = ["| kernel | family | counter | dispatches | average per dispatch |", "|---|---|---|---:|---:|"]
    for d in dirs:
        for name, cs in sorted(pmc_by_kernel(d).items()):
            for c, (avg, n) in sorted(cs.items()):
                out.append(f"| {short(name)} | {family(name) or '-'} | {c} | {n} | {avg:.1f} |")
    return out


def _family_avg(dirname, counter):
    """{family: average counter value per dispatch} over the family's kernels."""
    sums = collections.defaultdict(lambda: [0.0, 0])
    for name, cs in pmc_by_kernel(dirname).items():
        fam = family(name)
        if fam and counter in cs:
            avg, n = cs[counter]
            sums[fam][0] += avg * n
            sums[fam][1] += n
    return {f: s / n for f, (s, n) in sums.items() if n}


def traffic(fetch, write, copy_fetch, copy_write, copy_bytes, leg):
    cf = _family_avg(copy_fetch, "FETCH_SIZE")["copy"]
    cw = _family_avg(copy_write, "WRITE_SIZE")["copy"]
    read_scale, write_scale = copy_bytes / cf, copy_bytes / cw  # bytes per counter unit
    f, w = _family_avg(fetch, "FETCH_SIZE"), _family_avg(write, "WRITE_SIZE")
    fams = {}
    for fam in sorted(set(f) & set(w)):
        rd, wr = f[fam] * read_scale, w[fam] * write_scale
        fams[fam] = {"read_bytes": round(rd), "write_bytes": round(wr), "bytes_per_launch": round(rd + wr)}
    lines = ["| family | FETCH_SIZE per launch | WRITE_SIZE per launch | HBM bytes read | HBM bytes written |",
             "|---|---:|---:|---:|---:|"]
    for fam, d in fams.items():
        lines.append(f"| {fam} | {f[fam]:.1f} | {w[fam]:.1f} | {d['read_bytes']} | {d['write_bytes']} |")
    lines += ["", f"Calibration (copy kernel, {copy_bytes} B each way per launch): FETCH_SIZE {cf:.1f}, "
                  f"WRITE_SIZE {cw:.1f} per launch -> {read_scale:.2f} B per FETCH_SIZE unit, "
                  f"{write_scale:.2f} B per WRITE_SIZE unit.", "",
              "```json",
              json.dumps({"traffic": {"leg": leg, "sources_sha256": sources_sha256(), "families": fams,
                                      "read_scale": read_scale, "write_scale": write_scale}}, indent=1),
              "```"]
    return lines


def load_traffic(profiles_dir, leg):
    """{family: bytes per launch} from the committed summaries for `leg`, or {}
    when none was taken on the current sources."""
    sha = sources_sha256()
    for p in sorted(glob.glob(os.path.join(profiles_dir, "*.md"))):
        with open(p) as fh:
            text = fh.read()
        for block in re.findall(r"```json\n(.*?)\n```", text, re.S):
            try:
                d = json.loads(block).get("traffic")
            except ValueError:
                continue
            if d and d.get("leg") == leg and d.get("sources_sha256") == sha:
                return {f: v["bytes_per_launch"] for f, v in d["families"].items()}
    return {}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    p = sub.add_parser("pmc")
    p.add_argument("dirs", nargs="+")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--leg", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        lines = stats_table(a.dir)
    elif a.cmd == "pmc":
        lines = pmc_table(a.dirs)
    else:
        lines = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.leg)
    sys.stdout.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
