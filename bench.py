#!/usr/bin/env python
"""Throughput of the fused split-step path on one MI355X.

Metric: screen-steps/s at N = 1024, complex64.  One screen-step is one
realization advanced through one diffraction + screen step, including the
synthesis (or evolution) of that step's screen.  A benchmark step is one pass
of the whole path over one batch:

  forward  (value): headline workload, 64 realizations x 8 fresh screens per
           step (t advances every step), screens synthesised inside the passes,
           ensemble moments accumulated (turpy_propagate + turpy_stats);
  fwd+bwd: the same with screen-plane checkpoints and the adjoint
           (turpy_propagate_backward, dL/du_in and dL/dphi);
  ar:      the N = 1024 autoregressive workload, one time step =
           turpy_evolve (8 screens x 16 pairs) + turpy_propagate from the
           stored spectra + turpy_stats (256 screen-steps);
  plain:   the same forward physics as one PyTorch op per kernel
           (torch.fft, elementwise exp and multiplies), screens materialised.

Before any timed step each plan's column-pass and synthesis strip widths are
measured by turpy_plan_tune (or taken from --tune-cache); `config.strip_widths`
and `tuning` report them.  Prints one JSON line.  Inputs are seeded and
synthetic and already resident in HBM when the timed region starts.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "screen-steps/s at N=1024 c64 (fwd, fwd+bwd) vs plain GPU; % HBM roofline"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--realizations", type=int, default=64)
    ap.add_argument("--only", choices=["all", "fwd", "fwdbwd", "fwdbwd_rev", "ar", "plain", "copy", "fwd_as",
                                       "uneven"],
                    default="all",
                    help="run one leg (profiling runs)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON strip-width cache: read when the file exists (its widths are then used without "
                         "measuring), written at the end")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=16, help="realization pairs in the oracle sample (about 20 s of CPU work)")
    return ap.parse_args()


def step_bytes(path, leg):
    """Minimum HBM bytes per benchmark step of each kernel family, following
    the pass schedule of turpy_propagate / turpy_propagate_backward for a
    shared source plane, synthesised (or stored-spectrum) screens, nonzero
    first and last distances and no subharmonics (the headline and AR
    workloads).  plane = one N x N complex64 field."""
    plane = path.n * path.n * 8
    r, p, m = path.realizations, (path.realizations + 1) // 2, path.num_screens
    moments = 4 * 4 * 2 * path.n * path.n  # four float accumulators, read and written
    ck = r if leg == "fwdbwd" else 0
    spec = p if leg == "ar" else 0  # stored spectra read by the synthesis
    out = {
        # source row transform (1 plane in, 1 out) and the final inverse row pass
        "row_plain": (2 + 2 * r) * plane,
        # column pass 0 diffracts the single shared source plane in place
        "col": (2 + 2 * r * m) * plane,
        # the first screen pass reads that one plane for every realization
        "row_fwd": (m * (2 * r + p + ck) - (r - 1)) * plane,
        "synth": m * (p + spec) * plane,
    }
    if leg in ("fwd", "ar"):
        out["stats"] = r * plane + moments
    if leg == "ar":
        out["evolve"] = 2 * p * m * plane
    if leg == "fwdbwd":
        # adjoint: first and last row passes (g in and out), M + 1 column passes,
        # M screen passes reading g, scratch and checkpoint, writing g and dL/dphi
        out["row_plain"] += 4 * r * plane
        out["col"] += (m + 1) * 2 * r * plane
        out["row_bwd"] = m * (3 * r + p) * plane + m * r * path.n * path.n * 4
        out["synth"] += m * p * plane
    if leg == "copy":
        return {"copy": 2 * r * plane}
    return out


def run_steps(torch, fn, first, steps):
    for i in range(steps):
        fn(first + i)
    torch.cuda.synchronize()


def measure(torch, fn, steps, warmup, binding, families, path, leg):
    """Warm-up, then one untimed pass with every kernel family bracketed by HIP
    events (the per-kernel table), then the timed region: `steps` steps with
    only the dominant family bracketed, on the stream its kernels run on.
    Returns (seconds per step, kernel table, dominant family)."""
    run_steps(torch, fn, 0, warmup)
    binding.profile_only(None)
    binding.profile(True)
    run_steps(torch, fn, warmup, steps)
    table = kernel_table(binding, families, steps, path, leg)
    binding.profile(False)
    timed = [f for f in table if "bytes_per_launch" in table[f]]
    dom = max(timed, key=lambda f: table[f]["total_ms"]) if timed else None
    binding.profile_only(dom)
    binding.profile(dom is not None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(torch, fn, warmup + steps, steps)
    t1 = time.perf_counter()
    if dom is not None:
        n, ms = binding.profile_read(dom)
        d = table[dom]
        d["timed_region_avg_us"] = 1e3 * ms / n
        d["timed_region_launches"] = n
    binding.profile(False)
    binding.profile_only(None)
    return (t1 - t0) / steps, table, dom


def kernel_table(binding, families, steps, path, leg):
    per_step = step_bytes(path, leg)
    out = {}
    for f in families:
        n, ms = binding.profile_read(f)
        if not n:
            continue
        e = {"launches": n, "avg_us": 1e3 * ms / n, "total_ms": ms}
        if f in per_step:
            e["bytes_per_launch"] = per_step[f] * steps / n
            e["GBps"] = e["bytes_per_launch"] / (e["avg_us"] * 1e-6) / 1e9
            e["frac_hbm"] = e["GBps"] / HBM_PEAK_GBPS
        out[f] = e
    return out


def roofline(table, dom, traffic):
    """Roofline entry of the dominant family: algorithmic bytes per launch over
    its average launch duration inside the timed region."""
    d = table[dom]
    us = d.get("timed_region_avg_us", d["avg_us"])
    gbps = d["bytes_per_launch"] / (us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": gbps / HBM_PEAK_GBPS, "traffic": traffic.get(dom),
            "bytes_per_launch": d["bytes_per_launch"], "avg_us": us}


def plain_forward(torch, plan, path, u0, seed, t, H, phi):
    """One PyTorch op per kernel: the paper's own formulation of Eq. 1."""
    plan.screens(seed, t, out=phi)
    u = u0.expand(path.realizations, path.n, path.n)
    for i in range(path.num_screens):
        u = torch.fft.ifft2(torch.fft.fft2(u) * H[i])
        u = u * torch.exp(1j * phi[:, i])
    if path.dz[-1] > 0:
        u = torch.fft.ifft2(torch.fft.fft2(u) * H[-1])
    return u


def fresnel_tables(torch, np, path, device):
    kh = np.fft.fftfreq(path.n) * path.n
    df = 1.0 / (path.n * path.dx)
    f2 = (kh[:, None] ** 2 + kh[None, :] ** 2) * df * df
    out = []
    for dz in path.dz:
        rev = -0.5 * (path.wavelength / path.n0) * dz * f2
        rev -= np.rint(rev)
        out.append(torch.from_numpy(np.exp(2j * np.pi * rev).astype(np.complex64)).to(device))
    return out


def cpu_baseline(w, pairs):
    """The FP64 oracle as it stands, on a bounded sample of the forward workload."""
    import numpy as np

    from oracle import propagate as opr
    from oracle import screens as osc
    path = w.path.with_(realizations=2 * pairs)
    u0 = w.source_field().astype(np.complex64).astype(np.complex128)
    t0 = time.perf_counter()
    phi = osc.phase_screens(path, w.seed, t=0)
    opr.propagate(u0, path, phi)
    dt = time.perf_counter() - t0
    ss = path.realizations * path.num_screens
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": ss / dt, "unit": "screen-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{path.realizations} realizations x {path.num_screens} screens of the forward workload "
                      f"at N={path.n} (synthesis + propagation), numpy float64, single thread, {dt:.1f} s "
                      f"on {cpu} ({os.cpu_count()} logical CPUs visible)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported by this build "
              f"(realizations shard without communication, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2604_07248_amd import api, binding, prof_summary, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    binding.lib()
    fams = ["row_fwd", "row_bwd", "row_plain", "col", "synth", "sh", "evolve", "stats", "finalize", "copy"]

    if args.tune_cache and os.path.exists(args.tune_cache):
        api.tune_cache_load(args.tune_cache)
    w = workloads.headline(args.realizations)
    path = w.path
    plan = api.Plan(path)
    # strip widths of the column pass and the synthesis: measured (or cached)
    # before any timed step
    t_tune = time.perf_counter()
    widths = plan.tune()
    t_tune = time.perf_counter() - t_tune
    u0 = torch.from_numpy(w.source_field().astype(np.complex64)).to(dev)
    u_out = torch.empty((path.realizations, path.n, path.n), dtype=torch.complex64, device=dev)
    moments = api.Moments(path.n, path.dx)
    ss_per_step = path.realizations * path.num_screens
    result = {"metric": METRIC, "unit": "screen-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
              "data": "synthetic (seeded Philox screens, Gaussian source)",
              "config": {"workload": w.name + " (N=1024 over 1 m, 1064 nm, 1.5 km, Cn2=2e-14, l0=5 mm, L0=20 m, "
                                              "8 fresh screens per step, W0=5 cm)",
                         "n": path.n, "realizations": path.realizations, "screens": path.num_screens,
                         "screen_steps_per_step": ss_per_step, "strip_widths": widths}}

    def fwd(i):
        plan.propagate(u0, seed=w.seed, t=i, out=u_out)
        moments.add(u_out)

    if args.only in ("all", "fwd"):
        sec, ktab, dom = measure(torch, fwd, args.steps, args.warmup, binding, fams, path, "fwd")
        result["value"] = ss_per_step / sec
        result["ms_per_step"] = 1e3 * sec
        result["kernels"] = ktab
        # whole-path effective bandwidth: every family's algorithmic bytes per step
        result["path_effective_GBps"] = sum(step_bytes(path, "fwd").values()) / sec / 1e9
        result["roofline"] = roofline(ktab, dom, prof_summary.load_traffic(os.path.join(ROOT, "profiles"), "fwd"))

    if args.only in ("all", "fwd_as"):
        # the same forward step with the angular-spectrum transfer function (Sec. 2.1)
        pas = path.with_(tf_kind=workloads.TF_ANGULAR_SPECTRUM)
        plan_as = api.Plan(pas)
        plan_as.tune()

        def fwd_as(i):
            plan_as.propagate(u0, seed=w.seed, t=i, out=u_out)
            moments.add(u_out)

        sec, ktab, dom = measure(torch, fwd_as, args.steps, args.warmup, binding, fams, pas, "fwd")
        result["fwd_angular_spectrum"] = {"value": ss_per_step / sec, "unit": "screen-steps/s",
                                          "ms_per_step": 1e3 * sec, "kernels": ktab, "dominant": dom}
        plan_as.close()

    if args.only in ("all", "fwdbwd"):
        ck = torch.empty((path.realizations, path.num_screens, path.n, path.n), dtype=torch.complex64, device=dev)

        def fwdbwd(i):
            out, c = plan.propagate(u0, seed=w.seed, t=i, out=u_out, checkpoints=ck)
            plan.propagate_backward(out, c, seed=w.seed, t=i)

        sec, ktab, dom = measure(torch, fwdbwd, args.steps, args.warmup, binding, fams, path, "fwdbwd")
        result["fwd_bwd"] = {"value": ss_per_step / sec, "unit": "screen-steps/s", "ms_per_step": 1e3 * sec,
                             "kernels": ktab, "dominant": dom,
                             "path_effective_GBps": sum(step_bytes(path, "fwdbwd").values()) / sec / 1e9}
        del ck

    if args.only in ("all", "fwdbwd_rev"):
        # the checkpoint-free adjoint: screen-plane fields rebuilt from u_out
        def fwdbwd_rev(i):
            out = plan.propagate(u0, seed=w.seed, t=i, out=u_out)
            plan.propagate_backward(out, None, seed=w.seed, t=i, u_out=out)

        sec, ktab, dom = measure(torch, fwdbwd_rev, args.steps, args.warmup, binding, fams, path, "fwdbwd")
        ck_bytes = path.realizations * path.num_screens * path.n * path.n * 8
        result["fwd_bwd_reversible"] = {"value": ss_per_step / sec, "unit": "screen-steps/s",
                                        "ms_per_step": 1e3 * sec, "kernels": ktab, "dominant": dom,
                                        "checkpoint_bytes_saved": ck_bytes - 2 * path.realizations * path.n * path.n * 8}

    if args.only in ("all", "ar"):
        w3 = workloads.config3()
        p3 = w3.path
        plan3 = api.Plan(p3)
        plan3.tune()
        spec = plan3.init_spectra(w3.seed)
        u3 = torch.from_numpy(w3.source_field().astype(np.complex64)).to(dev)
        o3 = torch.empty((p3.realizations, p3.n, p3.n), dtype=torch.complex64, device=dev)
        m3 = api.Moments(p3.n, p3.dx)
        ex = w3.extra

        def ar(i):
            plan3.evolve(spec, w3.seed, i + 1, ex["alpha"], ex["shift_x"], ex["shift_y"])
            plan3.propagate(u3, spectra=spec, out=o3)
            m3.add(o3)

        sec, ktab, dom = measure(torch, ar, args.steps, args.warmup, binding, fams, p3, "ar")
        # one AR step captured in a HIP graph, replayed with the time step in
        # device memory (the evolution draws fresh innovations every replay)
        t3 = torch.ones(1, dtype=torch.int32, device=dev)
        plan3.bind_time(t3)
        g3 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g3):
            ar(0)

        def ar_replay(i):
            t3.fill_(i + 1)
            g3.replay()

        run_steps(torch, ar_replay, 0, 2)
        t0 = time.perf_counter()
        run_steps(torch, ar_replay, 2, args.steps)
        sec_graph = (time.perf_counter() - t0) / args.steps
        plan3.bind_time(None)
        del g3
        ss3 = p3.realizations * p3.num_screens
        result["ar"] = {"value": ss3 / sec, "unit": "screen-steps/s", "ms_per_step": 1e3 * sec,
                        "workload": w3.name + " (32 sequences, alpha=0.99, shift 0.5 px/step)",
                        "seconds_for_1000_steps": 1000 * sec, "kernels": ktab, "dominant": dom,
                        "graph_replay_ms_per_step": 1e3 * sec_graph,
                        "graph_seconds_for_1000_steps": 1000 * sec_graph,
                        "path_effective_GBps": sum(step_bytes(p3, "ar").values()) / sec / 1e9}
        plan3.close()
        del spec

    if args.only in ("all", "uneven"):
        # serving mix: the first 64 instances of the uneven workload (N = 256..2048,
        # 5-20 screens, three subharmonic levels, one realization each) in one
        # batch call, against the same instances run one plan after another
        inst = [x.path for x in workloads.uneven_batch()[:64]]
        batch = api.Batch(inst)
        t_bt = time.perf_counter()
        batch.tune()  # one measurement per (N, batch class); the plans below start from the cache
        t_bt = time.perf_counter() - t_bt
        srcs = [torch.from_numpy(workloads.gaussian_source(p.n, p.dx, p.n * p.dx / 8).astype(np.complex64))[None]
                for p in inst]
        ub = batch.pack(srcs)
        uo = torch.empty_like(ub)
        plans = [api.Plan(p) for p in inst]
        srcs = [x.to(dev) for x in srcs]
        outs = batch.unpack(uo)
        ss_u = sum(p.num_screens for p in inst)

        def one_call(i):
            batch.propagate(ub, seed=5, t=i, out=uo)

        def one_by_one(i):
            for k, pl in enumerate(plans):
                pl.propagate(srcs[k], seed=api.Batch.instance_seed(5, k), t=i, out=outs[k])

        res = {}
        for name, fn in (("batch", one_call), ("sequential", one_by_one)):
            run_steps(torch, fn, 0, 2)
            k = max(3, args.steps // 10)
            t0 = time.perf_counter()
            run_steps(torch, fn, 2, k)
            res[name] = (time.perf_counter() - t0) / k
        # the same call captured once in a HIP graph, replayed with the time
        # step read from device memory
        t_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        batch.bind_time(t_dev)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            batch.propagate(ub, seed=5, t=0, out=uo)

        def replay(i):
            t_dev.fill_(i)
            graph.replay()

        run_steps(torch, replay, 0, 2)
        k = max(3, args.steps // 10)
        t0 = time.perf_counter()
        run_steps(torch, replay, 2, k)
        res["graph"] = (time.perf_counter() - t0) / k
        batch.bind_time(None)
        del graph
        result["uneven_batch"] = {
            "value": ss_u / res["batch"], "unit": "screen-steps/s", "instances": len(inst),
            "instances_per_s": len(inst) / res["batch"], "ms_per_call": 1e3 * res["batch"],
            "sequential_ms": 1e3 * res["sequential"], "speedup_vs_sequential": res["sequential"] / res["batch"],
            "graph_replay_ms": 1e3 * res["graph"], "graph_instances_per_s": len(inst) / res["graph"],
            "workload": "first 64 serving-mix instances (N 256-2048, 5-20 screens, 3 subharmonic levels, R=1)",
            "tune_seconds": t_bt}
        for pl in plans:
            pl.close()
        batch.close()

    if args.only in ("all", "plain"):
        H = fresnel_tables(torch, np, path, dev)
        phi = torch.empty((path.realizations, path.num_screens, path.n, path.n), dtype=torch.float32, device=dev)

        def plain(i):
            u = plain_forward(torch, plan, path, u0, w.seed, i, H, phi)
            moments.add(u)

        k = max(2, args.steps // 5)
        run_steps(torch, plain, 0, 2)
        t0 = time.perf_counter()
        run_steps(torch, plain, 2, k)
        sec = (time.perf_counter() - t0) / k
        # same screens, same physics: report the agreement of the two versions
        fused = plan.propagate(u0, seed=w.seed, t=0)
        ref = plain_forward(torch, plan, path, u0, w.seed, 0, H, phi)
        diff = float(torch.linalg.vector_norm(fused - ref) / torch.linalg.vector_norm(ref))
        result["plain_gpu"] = {"value": ss_per_step / sec, "unit": "screen-steps/s", "ms_per_step": 1e3 * sec,
                               "kind": "one PyTorch op per kernel (torch.fft + elementwise), same screens",
                               "rel_l2_vs_fused": diff}
        if "value" in result:
            result["speedup_vs_plain"] = result["value"] / result["plain_gpu"]["value"]
        del phi, H

    if args.only == "copy":
        # calibration: the library's plain copy kernel (no screens, no diffraction) of known size
        pc = workloads.Path(n=path.n, dx=path.dx, wavelength=path.wavelength, dz=(0.0,), cn2dz=(),
                            realizations=path.realizations)
        planc = api.Plan(pc)
        src = torch.empty_like(u_out).copy_(u0.expand_as(u_out))
        _, ktab, _ = measure(torch, lambda i: planc.propagate(src, out=u_out), args.steps, args.warmup, binding,
                             fams, pc, "copy")
        result["copy"] = ktab
        result["value"] = 0.0

    result["tuning"] = {"headline_seconds": t_tune, "cache": api.tune_cache()}
    if args.tune_cache:
        api.tune_cache_save(args.tune_cache)
    if args.only == "all" and not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_pairs)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
