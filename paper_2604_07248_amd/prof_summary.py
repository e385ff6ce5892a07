"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_2604_07248_amd.prof_summary stats DIR
        Markdown table of a `--kernel-trace --stats --output-format csv` run.
    python -m paper_2604_07248_amd.prof_summary pmc DIR [DIR ...]
        Per-kernel average of every counter of `--pmc ... --output-format csv` runs.
    python -m paper_2604_07248_amd.prof_summary report --bench BENCH_JSON [--out profiles]
        All summaries of the standard profiling runs under --root (the $OUT of their commands).
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
        if p.endswith((".hip", ".hpp", ".h", ".cpp")):
            h.update(os.path.basename(p).encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def family(kernel_name):
    """turpy_profile family of a kernel, from its demangled name."""
    n = kernel_name
    if "turpy::" not in n:
        return None  # runtime and PyTorch kernels
    m = re.search(r"row_(?:pair|pass)_kernel<(\d+), (\d+), (true|false)", n)
    if m:
        if m.group(2) == "0":
            return "row_plain"
        return "row_bwd" if m.group(3) == "true" else "row_fwd"
    m = re.search(r"row_pass_group_kernel<(\d+), (\d+)>", n)
    if m:
        return "row_plain" if m.group(2) == "0" else "row_fwd"
    if "_group_bwd_kernel" in n:
        return "row_bwd"
    if "row_relay" in n or "row_pair_group_kernel" in n:
        return "row_fwd"
    for key, fam in (("row_moments_kernel", "row_moments"), ("col_pass", "col"), ("synth_", "synth"),
                     ("sh_kernel", "sh"), ("sh_group_kernel", "sh"), ("evolve_kernel", "evolve"),
                     ("stats_kernel", "stats"), ("finalize_kernel", "finalize"), ("copy_kernel", "copy"),
                     ("sum_planes_kernel", "sum"), ("noise_kernel", "noise"), ("nonfinite_kernel", "nonfinite"),
                     ("recv_row_in", "recv_row"), ("recv_col_grad", "recv_col_grad"), ("recv_col", "recv_col"),
                     ("recv_row_grad", "recv_row_grad"), ("recv_reduce", "recv_reduce")):
        if key in n:
            return fam
    return None


def short(kernel_name):
    n = re.sub(r"turpy::\(anonymous namespace\)::", "", kernel_name)
    n = re.sub(r"^void ", "", n)
    n = re.sub(r"\([^()]*\)$", "", n)  # the argument list
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


PRE = "cd /tmp && export TMPDIR=/tmp && R=<repository root> && OUT=<output directory>"
TUNE = "--tune-cache $OUT/tune.json --no-cpu-baseline"

# The standard profiling runs: (directory under $OUT, bench.py arguments).
TRACES = {
    "prof_fwd": "--only fwd --steps 10 --warmup 2",
    "prof_fwdbwd": "--only fwdbwd --steps 5 --warmup 2",
    "prof_ar": "--only ar --steps 10 --warmup 2",
    "prof_uneven": "--only uneven --uneven-waves 1 --steps 25 --warmup 1",
}
PMC_SQ = ("SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_LDS "
          "GRBM_GUI_ACTIVE")
PMC_STALL = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS "
             "SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_LDS GRBM_GUI_ACTIVE TA_BUSY_avr TCP_PENDING_STALL_CYCLES_sum "
             "TCP_TCP_TA_ADDR_STALL_CYCLES_sum")


def _ev(fams, tab):
    return ", ".join(f"{f} {tab[f]['avg_us']:.1f} us" for f in fams if f in tab)


def _trace_cmd(d):
    return ["    rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/" + d + " -o t -- \\",
            f"        python $R/bench.py {TRACES[d]} {TUNE}"]


def _pmc_cmd(counters, d, leg):
    return [f"    timeout -s KILL 120 rocprofv3 --pmc {counters} --output-format csv -d $OUT/{d} -o p -- \\",
            f"        python $R/bench.py --only {leg} --steps 3 --warmup 1 {TUNE}"]


def report(out_dir, bench_json, root):
    """Write the committed summaries of the standard profiling runs (the
    commands are printed in each file) into out_dir."""
    with open(bench_json) as fh:
        b = json.load(fh)
    j = lambda *a: os.path.join(root, *a)
    head = ["Commands (one MI355X; the profiler writes its temporary files under /tmp).  The default",
            "benchmark run writes the launch configuration its tuner chose; the profiled runs read it back,",
            "so that their traces hold no tuning launches:", "",
            f"    {PRE}", "    python $R/bench.py --tune-cache $OUT/tune.json > $OUT/bench.json"]
    # forward kernel trace
    rows = stats_table(j("prof_fwd"))
    d = b["roofline"]
    dom_rows = [r for r in rows[2:] if f"| {d['kernel']} |" in r]
    lines = ["# Kernel trace: forward headline workload (N=1024, R=64, M=8, fresh screens)", ""] + head + \
        _trace_cmd("prof_fwd") + [
        "", "Summary: `python -m paper_2604_07248_amd.prof_summary stats $OUT/prof_fwd`.  The run covers",
        "22 forward steps: 2 warm-up, 10 with every family bracketed by events, 10 timed.  Durations in",
        "microseconds.", ""] + rows + [
        "", "HIP-event averages measured inside `bench.py` (default run: 5 warm-up, 50 profiled and 50 timed "
        "steps): " + _ev(["row_fwd", "col", "synth", "row_moments", "row_plain"], b["kernels"]) + ".", "",
        f"Roofline line of that run: dominant family `{d['kernel']}`, {d['bytes_per_launch']:.0f} algorithmic "
        f"bytes per launch over {d['avg_us']:.1f} us = {d['achieved']:.0f} GB/s = {100 * d['frac']:.1f} % of "
        f"8 TB/s; the trace's average for that family is "
        f"{' / '.join(r.split('|')[5].strip() for r in dom_rows)} us."]
    _write(out_dir, "fwd_h1_n1024_r64_m8_kernel_stats.md", lines)
    # forward + adjoint, AR and serving-mix kernel traces
    for d_, name, title, tab, fams in (
            ("prof_fwdbwd", "fwdbwd_h1_n1024_r64_m8_kernel_stats.md",
             "forward + adjoint, headline workload (N=1024, R=64, M=8, screen checkpoints)",
             b["fwd_bwd"]["kernels"], ["row_fwd", "row_bwd", "col", "synth", "row_plain", "sum"]),
            ("prof_ar", "ar_c3_n1024_r32_m8_kernel_stats.md",
             "AR workload (N=1024, 32 sequences, M=8; the evolution fused into the synthesis)",
             b["ar"]["kernels"], ["row_fwd", "col", "synth", "row_moments", "row_plain"]),
            ("prof_uneven", "uneven_c5_serving_mix_kernel_stats.md",
             "serving mix (one wave of 256 instances, N 256-2048, R=1; grouped launches)", None, [])):
        lines = [f"# Kernel trace: {title}", ""] + head + _trace_cmd(d_) + [
            "", f"Summary: `python -m paper_2604_07248_amd.prof_summary stats $OUT/{d_}`.", ""]
        lines += stats_table(j(d_))
        if tab:
            lines += ["", "HIP-event averages inside `bench.py` (default run): " + _ev(fams, tab) + "."]
        _write(out_dir, name, lines)
    # HBM traffic of the forward and the forward + adjoint legs
    for leg, title in (("fwd", "forward"), ("fwdbwd", "forward + adjoint")):
        lines = [f"# HBM traffic per launch: {title}, headline workload (N=1024, R=64, M=8)", "",
                 "Commands (one counter per run; the copy runs calibrate the counters with the library's copy",
                 "kernel moving 512 MiB each way per launch):", "", f"    {PRE}"]
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            for lg in (leg, "copy"):
                lines += _pmc_cmd(c, f"pmc_{c}_{lg}", lg)
        lines += ["", "Summary: `python -m paper_2604_07248_amd.prof_summary traffic --fetch "
                  f"$OUT/pmc_FETCH_SIZE_{leg} --write $OUT/pmc_WRITE_SIZE_{leg} --copy-fetch "
                  "$OUT/pmc_FETCH_SIZE_copy --copy-write $OUT/pmc_WRITE_SIZE_copy --copy-bytes "
                  f"536870912 --leg {leg}`.", "",
                  "Averages over every launch of a family (the column family includes the one-plane pass 0, the",
                  "row-plain family the one-plane transforms).  On gfx950 almost every read is a 128-byte",
                  "request, which the FETCH_SIZE expression counts as 64 bytes: the copy calibration sets the",
                  "bytes per counter unit.", ""]
        lines += traffic(j(f"pmc_FETCH_SIZE_{leg}"), j(f"pmc_WRITE_SIZE_{leg}"), j("pmc_FETCH_SIZE_copy"),
                         j("pmc_WRITE_SIZE_copy"), 536870912, leg)
        _write(out_dir, f"{leg}_h1_n1024_r64_m8_hbm_traffic.md", lines)
    for leg, title in (("fwd", "forward"), ("fwdbwd", "forward + adjoint")):
        _sq_summary(out_dir, j, leg, title)
        _stall_summary(out_dir, j, leg, title)


def _sq_summary(out_dir, j, leg, title):
    """VALU and wave counters of one leg."""
    d = f"pmc_sq_{leg}"
    if not os.path.isdir(j(d)):
        return
    sq = pmc_by_kernel(j(d))
    lines = [f"# Wave and VALU counters: {title}, headline workload (N=1024, R=64, M=8)", "", "Command:", "",
             f"    {PRE}"] + _pmc_cmd(PMC_SQ, d, leg) + [
             "", f"Summary: `python -m paper_2604_07248_amd.prof_summary pmc $OUT/{d}` (per-dispatch",
             "averages).  VALU busy = SQ_INSTS_VALU x 4 cycles (a wave64 FP32 instruction on a 16-lane SIMD) /",
             "(1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs).", "",
             "| family | waves | VALU instr per wave | LDS instr per wave | kernel cycles | VALU busy |",
             "|---|---:|---:|---:|---:|---:|"]
    for name, cs in sorted(sq.items(), key=lambda kv: family(kv[0]) or "z"):
        fam = family(name)
        if not fam:
            continue
        waves, valu, lds = cs["SQ_WAVES"][0], cs["SQ_INSTS_VALU"][0], cs["SQ_INSTS_LDS"][0]
        cyc = cs["GRBM_GUI_ACTIVE"][0] / 8
        lines.append(f"| {fam} | {waves:.0f} | {valu / waves:.0f} | {lds / waves:.0f} | {cyc:.0f} | "
                     f"{100 * valu * 4 / (1024 * cyc):.0f} % |")
    lines += ["", "Full table:", ""] + pmc_table([j(d)])
    _write(out_dir, f"{leg}_h1_n1024_r64_m8_sq_counters.md", lines)


def _stall_summary(out_dir, j, leg, title):
    """Stall and occupancy counters of one leg."""
    d = f"pmc_stall_{leg}"
    if not os.path.isdir(j(d)):
        return
    st = pmc_by_kernel(j(d))
    lines = [f"# Stall and occupancy counters: {title}, headline workload (N=1024, R=64, M=8)", "", "Command:", "",
             f"    {PRE}"] + _pmc_cmd(PMC_STALL, d, leg) + [
             "", f"Summary: `python -m paper_2604_07248_amd.prof_summary pmc $OUT/{d}` (per-dispatch",
             "averages).  With c = GRBM_GUI_ACTIVE / 8 (kernel cycles; the counter adds the 8 XCDs): waves",
             "resident per CU = 4 SQ_WAVE_CYCLES / (256 c) (the SQ cycle counters count 4-cycle units); wait",
             "fractions = SQ_WAIT_ANY and SQ_WAIT_INST_ANY over SQ_WAVE_CYCLES; LDS bank conflicts per",
             "LDS-active cycle = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS; TA busy = TA_BUSY_avr / c.", "",
             "| family | waves per CU | wait any | wait inst | LDS conflicts per LDS cycle | TA busy | "
             "TCP pending-stall cycles |", "|---|---:|---:|---:|---:|---:|---:|"]
    for name, cs in sorted(st.items(), key=lambda kv: family(kv[0]) or "z"):
        fam = family(name)
        if not fam:
            continue
        wc = max(cs["SQ_WAVE_CYCLES"][0], 1.0)
        c = max(cs["GRBM_GUI_ACTIVE"][0] / 8, 1.0)
        lds = max(cs["SQ_ACTIVE_INST_LDS"][0], 1.0)
        lines.append(f"| {fam} | {4 * wc / (256 * c):.1f} | {100 * cs['SQ_WAIT_ANY'][0] / wc:.0f} % | "
                     f"{100 * cs['SQ_WAIT_INST_ANY'][0] / wc:.0f} % | {cs['SQ_LDS_BANK_CONFLICT'][0] / lds:.2f} | "
                     f"{100 * cs['TA_BUSY_avr'][0] / c:.0f} % | {cs['TCP_PENDING_STALL_CYCLES_sum'][0]:.0f} |")
    lines += ["", "Full table:", ""] + pmc_table([j(d)])
    _write(out_dir, f"{leg}_h1_n1024_r64_m8_stall_counters.md", lines)


def _write(out_dir, name, lines):
    with open(os.path.join(out_dir, name), "w") as fh:
        fh.write("\n".join(lines) + "\n")


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
    r = sub.add_parser("report", help="write the committed summaries of the standard runs")
    r.add_argument("--bench", required=True, help="bench.py JSON of the same sources")
    r.add_argument("--out", default="profiles")
    r.add_argument("--root", required=True, help="the output directory of the runs ($OUT)")
    a = ap.parse_args(argv)
    if a.cmd == "report":
        report(a.out, a.bench, a.root)
        return
    if a.cmd == "stats":
        lines = stats_table(a.dir)
    elif a.cmd == "pmc":
        lines = pmc_table(a.dirs)
    else:
        lines = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.leg)
    sys.stdout.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
