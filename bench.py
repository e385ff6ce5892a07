#!/usr/bin/env python
"""Throughput of the fused split-step path on one MI355X.

Metric: screen-steps/s at N = 1024, complex64.  One screen-step is one
realization advanced through one diffraction + screen step, including the
synthesis (or evolution) of that step's screen.  A benchmark step is one pass
of the whole path over one batch:

  forward  (value): headline workload, 64 realizations x 8 fresh screens per
           step (t advances every step), screens synthesised inside the passes,
           ensemble moments taken inside the final row pass (turpy_propagate
           on a plan bound to the moment sums);
  fwd+bwd: the same with screen-plane checkpoints (fields and the screens'
           column halves) and the adjoint (turpy_propagate_backward, dL/du_in
           of the shared source and dL/dphi);
  ar:      the N = 1024 autoregressive workload, one time step =
           turpy_evolve_propagate (the AR step of 8 screens x 16 pairs fused
           into the propagation's screen synthesis, moments inside the final
           row pass; 256 screen-steps); also timed as turpy_evolve +
           turpy_propagate;
  plain:   the same physics one op per kernel: Philox normals (turpy_noise),
           torch elementwise ops and torch.fft for the screens and Eq. 1,
           forward and forward + backward (torch autograd).
The FP64 oracle is timed first, on the host cores (one and all), before the
GPU is touched (`cpu_baseline`); the forward step's error against it is
`oracle_rel_l2`.

Before any timed step each plan's launch configuration (strip widths and radix
plans of the column pass and the synthesis, occupancy hints of the screen row
passes) is measured by turpy_plan_tune (or taken from --tune-cache);
`config.launch_config` and `tuning` report them.  Prints one JSON line.  Inputs are seeded and
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
                    help="JSON tuning cache: read when the file exists (its choices are then used without "
                         "measuring), written at the end")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=16, help="realization pairs in the oracle sample (about 20 s of CPU work)")
    ap.add_argument("--uneven-waves", type=int, default=16,
                    help="waves of 256 serving-mix instances in the uneven leg (16: all 4096; fewer for profiling runs)")
    return ap.parse_args()


def step_bytes(path, leg):
    """Minimum HBM bytes per benchmark step of each kernel family, following
    the pass schedules of turpy_propagate and of the two adjoints for a shared
    source plane, synthesised (or stored-spectrum) screens, nonzero first and
    last distances and no subharmonics (the headline and AR workloads).  The
    adjoints return the gradient of the shared source (summed over
    realizations right after screen 0).  plane = one N x N complex64 field.
    legs: fwd (with moments), ar, fwdbwd (checkpoints), fwdbwd_rev
    (checkpoint-free adjoint), copy."""
    plane = path.n * path.n * 8
    r, p, m = path.realizations, (path.realizations + 1) // 2, path.num_screens
    moments = 4 * 4 * 2 * path.n * path.n  # four float accumulators, read and written
    gphi = r * path.n * path.n * 4          # dL/dphi of one screen, float
    if leg == "copy":
        return {"copy": 2 * r * plane}
    ck = r if leg == "fwdbwd" else 0
    # ar: the synthesis reads each screen's stored spectra, writes them back
    # evolved and writes the scratch (the evolution fused into it)
    spec = 2 * p if leg == "ar" else 0
    out = {
        # source row transform (1 plane in, 1 out)
        "row_plain": 2 * plane,
        # column pass 0 diffracts the single shared source plane in place
        "col": (2 + 2 * r * m) * plane,
        # the first screen pass reads that one plane for every realization
        "row_fwd": (m * (2 * r + p + ck) - (r - 1)) * plane,
        "synth": m * (p + spec) * plane,
    }
    if leg in ("fwd", "ar"):
        # the final inverse row pass, with the moments taken inside it
        out["row_moments"] = 2 * r * plane + moments
    else:
        out["row_plain"] += 2 * r * plane
    if leg == "fwdbwd":
        # first row pass (g in and out), M column passes on R planes, M screen
        # passes reading g, scratch and checkpoint and writing g and dL/dphi;
        # after screen 0 the R gradients are summed into one plane, which
        # column pass 0 and the last row pass carry alone
        out["row_plain"] += (2 * r + 2) * plane
        out["col"] += (2 * r * m + 2) * plane
        out["row_bwd"] = m * (3 * r + p) * plane + m * gphi
        out["sum"] = (r + 1) * plane
        # the screens' column halves are kept with the checkpoints: the
        # forward synthesis writes them there, the adjoint synthesises none
    if leg == "fwdbwd_rev":
        # two chains (gradient and rebuilt field): first row and column pass on
        # both; per screen the field chain reads its field and the scratch and
        # writes the rebuilt field at the screen (and, except at screen 0, its
        # continuation), the gradient chain reads g, the scratch and that field
        # and writes g and dL/dphi; both chains' column passes except after
        # screen 0, where the gradient is summed into one plane first
        out["row_plain"] += (4 * r + 2) * plane
        out["col"] += (4 * r * m + 2) * plane
        out["row_bwd"] = (m * (6 * r + 2 * p) - r) * plane + m * gphi
        out["sum"] = (r + 1) * plane
        out["synth"] += m * p * plane
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


def roofline(table, dom, traffic, path, leg, sec):
    """Roofline entry of the dominant family: algorithmic bytes per launch over
    its average launch duration inside the timed region.  `step` holds the
    whole step's figure: every family's algorithmic bytes per step over the
    measured time per step (the figure the 60 % target is read against)."""
    d = table[dom]
    us = d.get("timed_region_avg_us", d["avg_us"])
    gbps = d["bytes_per_launch"] / (us * 1e-6) / 1e9
    step = sum(step_bytes(path, leg).values())
    return {"bound": "hbm", "kernel": dom, "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": gbps / HBM_PEAK_GBPS, "traffic": traffic.get(dom),
            "bytes_per_launch": d["bytes_per_launch"], "avg_us": us,
            "step": {"bytes": step, "ms": 1e3 * sec, "achieved": step / sec / 1e9,
                     "frac": step / sec / 1e9 / HBM_PEAK_GBPS}}


def psd_amplitudes(np, path):
    """Per-screen spectral amplitude sqrt(W(f)) df in radians (Eq. S16-S18,
    frequencies in cycles/m, DC zero), float32 [M][N][N]: the per-op
    baseline's weighting table, computed once."""
    n = path.n
    kh = np.fft.fftfreq(n) * n
    df = 1.0 / (n * path.dx)
    f2 = (kh[:, None] ** 2 + kh[None, :] ** 2) * df * df
    k = 2 * np.pi * path.n0 / path.wavelength
    fm2 = (1.0 / path.l0) ** 2 if path.l0 > 0 else np.inf
    f02 = (1.0 / path.L0) ** 2 if np.isfinite(path.L0) and path.L0 > 0 else 0.0
    f2s = np.where(f2 > 0, f2, 1.0)
    out = []
    for c in path.cn2dz:
        w = 0.023 * 0.423 * k * k * c * np.exp(-f2s / fm2) / (f2s + f02) ** (11.0 / 6.0)
        a = np.sqrt(w) * df
        a[0, 0] = 0.0
        out.append(a.astype(np.float32))
    return np.stack(out)


def plain_screens(torch, api, path, seed, t, amp, phi):
    """Screens one op per kernel: Philox normals (turpy_noise), PSD weighting,
    unnormalised inverse FFT, real/imaginary split, piston removal."""
    pairs = (path.realizations + 1) // 2
    for s in range(path.num_screens):
        c = api.noise(path.n, pairs, seed, t=t, tag=1, screen=s) * amp[s]
        z = torch.fft.ifft2(c, norm="forward")
        re_im = torch.stack((z.real, z.imag), dim=1).reshape(2 * pairs, path.n, path.n)[:path.realizations]
        phi[:, s] = re_im - re_im.mean(dim=(-1, -2), keepdim=True)
    return phi


def plain_propagate(torch, path, u0, H, phi):
    """Eq. 1 one PyTorch op per kernel (the paper's own formulation)."""
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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown CPU"


def _oracle_pair(args):
    """One realization pair of the forward workload through the oracle."""
    import numpy as np

    from oracle import propagate as opr
    from oracle import screens as osc
    path, seed, pair, u0 = args
    m = path.num_screens
    phi = np.empty((2, m, path.n, path.n))
    for s in range(m):
        phi[0, s], phi[1, s] = osc.split_pair(osc.complex_screen(path, seed, 0, pair, s))
    return opr.propagate(u0, path.with_(realizations=2), phi)[0]


def cpu_baseline(w, pairs):
    """The FP64 oracle as it stands, timed on the host cores before the GPU is
    touched: a bounded sample of the forward workload (`pairs` realization
    pairs, t = 0) on one core and on every core of the process's CPU share
    (one process per pair), and the N = 128 five-screen workload in full on
    one core.  Returns (record, the sample's fields)."""
    import multiprocessing as mp

    import numpy as np

    from oracle import propagate as opr
    from oracle import screens as osc
    from paper_2604_07248_amd import workloads
    path = w.path.with_(realizations=2 * pairs)
    u0 = w.source_field().astype(np.complex64).astype(np.complex128)
    t0 = time.perf_counter()
    phi = osc.phase_screens(path, w.seed, t=0)
    fields, _ = opr.propagate(u0, path, phi)
    dt1 = time.perf_counter() - t0
    del phi
    cores = max(1, min(16, len(os.sched_getaffinity(0)), pairs))
    ctx = mp.get_context("fork")  # the GPU is not initialised yet
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        outs = pool.map(_oracle_pair, [(path, w.seed, j, u0) for j in range(pairs)], chunksize=1)
    dtn = time.perf_counter() - t0
    agree = max(float(np.max(np.abs(o - fields[2 * j:2 * j + 2]))) for j, o in enumerate(outs))
    del outs
    c1 = workloads.config1()
    t0 = time.perf_counter()
    opr.propagate(c1.source_field().astype(np.complex128), c1.path, osc.phase_screens(c1.path, c1.seed))
    dt_c1 = time.perf_counter() - t0
    ss = path.realizations * path.num_screens
    cpu = _cpu_model()
    rec = {"value": ss / dtn, "unit": "screen-steps/s", "cores": cores, "kind": "oracle",
           "sample": f"{path.realizations} realizations x {path.num_screens} screens of the forward workload at "
                     f"N={path.n} (synthesis + propagation, t=0), numpy float64, {cores} processes (one pair each) "
                     f"in {dtn:.1f} s on {cpu}",
           "single_core": {"value": ss / dt1, "seconds": dt1},
           "all_core_seconds": dtn, "all_core_max_abs_diff_vs_single": agree,
           "config1_full": {"workload": c1.name, "seconds": dt_c1,
                            "screen_steps_per_s": c1.path.realizations * c1.path.num_screens / dt_c1, "cores": 1},
           "cpu_model": cpu, "logical_cpus_visible": os.cpu_count()}
    return rec, fields


def plain_instance(torch, api, path, seed, t, u0, tabs, grad=False):
    """One serving-mix instance one op per kernel: Philox normals
    (turpy_noise), PSD weighting, unnormalised inverse FFT; the three Lane
    subharmonic levels as two small matrix products per screen (their
    coefficients drawn by torch); piston; then Eq. 1 with torch.fft.  With
    grad, the backward through torch's autograd (source and screens)."""
    H, amp, shamp, ey, ex = tabs
    n, m = path.n, path.num_screens
    phi = torch.empty((1, m, n, n), dtype=torch.float32, device=u0.device)
    for s in range(m):
        z = torch.fft.ifft2(api.noise(n, 1, seed, t=t, tag=1, screen=s) * amp[s], norm="forward")[0]
        c = torch.randn((3, 3, 3), dtype=torch.complex64, device=u0.device) * shamp[s]
        for lv in range(3):
            z = z + ey[lv].T @ c[lv] @ ex[lv]
        phi[0, s] = z.real - z.real.mean()
    u = u0.detach().requires_grad_(grad)
    ph = phi.requires_grad_(grad)
    out = plain_propagate(torch, path, u, H, ph)
    if grad:
        torch.autograd.backward(out, grad_tensors=out.detach())
    return out


def plain_instance_tables(torch, np, path, dev):
    """Transfer functions, PSD amplitudes, subharmonic amplitudes (centre
    zero) and phasors exp(2 pi i (0, +-1) df/3^p x) of one instance."""
    H = fresnel_tables(torch, np, path, dev)
    amp = torch.from_numpy(psd_amplitudes(np, path)).to(dev)
    n, dx = path.n, path.dx
    df = 1.0 / (n * dx)
    k = 2 * np.pi * path.n0 / path.wavelength
    x = (np.arange(n) - n // 2) * dx
    off = np.array([-1.0, 0.0, 1.0])
    shamp = np.zeros((path.num_screens, 3, 3, 3))
    ey = []
    for lv in range(3):
        dfp = df / 3 ** (lv + 1)
        f2 = (off[:, None] ** 2 + off[None, :] ** 2) * dfp * dfp
        for s, c in enumerate(path.cn2dz):
            w = 0.023 * 0.423 * k * k * c * np.exp(-f2 * path.l0 ** 2) / (f2 + path.L0 ** -2) ** (11.0 / 6.0)
            a = np.sqrt(w) * dfp
            a[1, 1] = 0.0
            shamp[s, lv] = a
        ey.append(torch.from_numpy(np.exp(2j * np.pi * off[:, None] * dfp * x[None, :]).astype(np.complex64)).to(dev))
    shamp = torch.from_numpy(shamp.astype(np.float32)).to(dev)
    return H, amp, shamp, ey, ey


def uneven_leg(torch, np, api, workloads, args, dev, wave=256):
    """The serving mix at full size: 4096 path instances (N = 256..2048,
    5-20 screens, three subharmonic levels, one realization each), run in
    memory-budgeted waves of `wave` instances, each wave one turpy_batch call
    (forward; forward + backward with checkpoints), also replayed from HIP
    graphs; the plain one-op-per-kernel version is timed on the first wave."""
    inst = [x.path for x in workloads.uneven_batch()][:wave * args.uneven_waves]
    waves = [inst[i:i + wave] for i in range(0, len(inst), wave)]
    t0 = time.perf_counter()
    batches = [api.Batch(wv) for wv in waves]
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    for bt in batches:
        bt.tune()
    t_tune = time.perf_counter() - t0
    srcs = []
    for wv, bt in zip(waves, batches):
        fields = [torch.from_numpy(workloads.gaussian_source(p.n, p.dx, p.n * p.dx / 8).astype(np.complex64))[None]
                  for p in wv]
        srcs.append(bt.pack(fields))
    out = torch.empty(max(bt.total for bt in batches), dtype=torch.complex64, device=dev)
    ss = sum(p.num_screens for p in inst)
    px = sum(p.n * p.n * p.num_screens for p in inst)

    def fwd(i):
        for bt, src in zip(batches, srcs):
            bt.propagate(src, seed=5, t=i, out=out[:bt.total])

    res = {}
    k = max(2, args.steps // 25)
    run_steps(torch, fwd, 0, 1)
    t0 = time.perf_counter()
    run_steps(torch, fwd, 1, k)
    res["fwd"] = (time.perf_counter() - t0) / k
    # each wave's call captured once in a HIP graph, replayed with the time step
    # read from device memory
    t_dev = torch.zeros(1, dtype=torch.int32, device=dev)
    graphs = []
    for bt, src in zip(batches, srcs):
        bt.bind_time(t_dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            bt.propagate(src, seed=5, t=0, out=out[:bt.total])
        graphs.append(g)

    def replay(i):
        t_dev.fill_(i)
        for g in graphs:
            g.replay()

    run_steps(torch, replay, 0, 1)
    t0 = time.perf_counter()
    run_steps(torch, replay, 1, k)
    res["graph"] = (time.perf_counter() - t0) / k
    for bt in batches:
        bt.bind_time(None)
    del graphs

    # forward + backward, wave after wave, one checkpoint buffer reused
    ck = torch.empty(max(bt.ck_total for bt in batches), dtype=torch.complex64, device=dev)
    gin = torch.empty_like(out)
    gphi = torch.empty(ck.numel(), dtype=torch.float32, device=dev)

    def fwdbwd(i):
        for bt, src in zip(batches, srcs):
            o, c = bt.propagate(src, seed=5, t=i, out=out[:bt.total], checkpoints=ck[:bt.ck_total])
            bt.propagate_backward(o, c, seed=5, t=i, grad_in=gin[:bt.total], grad_screens=gphi[:bt.ck_total])

    run_steps(torch, fwdbwd, 0, 1)
    t0 = time.perf_counter()
    run_steps(torch, fwdbwd, 1, k)
    res["fwdbwd"] = (time.perf_counter() - t0) / k
    del ck, gin, gphi

    # plain version on the first wave
    first = waves[0]
    tabs = [plain_instance_tables(torch, np, p, dev) for p in first]
    u0s = [s.to(dev) for s in batches[0].unpack(srcs[0])]

    def plain(i, grad=False):
        for j, p in enumerate(first):
            plain_instance(torch, api, p, api.Batch.instance_seed(5, j), i, u0s[j], tabs[j], grad)

    plain(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain(1)
    torch.cuda.synchronize()
    res["plain_fwd_wave"] = time.perf_counter() - t0
    plain(0, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain(1, True)
    torch.cuda.synchronize()
    res["plain_fwdbwd_wave"] = time.perf_counter() - t0
    # the fused batch on the same first wave alone
    run_steps(torch, lambda i: batches[0].propagate(srcs[0], seed=5, t=i, out=out[:batches[0].total]), 0, 1)
    t0 = time.perf_counter()
    run_steps(torch, lambda i: batches[0].propagate(srcs[0], seed=5, t=i, out=out[:batches[0].total]), 1, k)
    res["fwd_wave"] = (time.perf_counter() - t0) / k
    ss_w = sum(p.num_screens for p in first)
    for bt in batches:
        bt.close()
    return {"value": ss / res["fwd"], "unit": "screen-steps/s", "instances": len(inst), "waves": len(waves),
            "wave_instances": wave, "ms_per_call": 1e3 * res["fwd"], "instances_per_s": len(inst) / res["fwd"],
            "pixel_screen_steps_per_s": px / res["fwd"],
            "graph_replay_ms": 1e3 * res["graph"], "graph_instances_per_s": len(inst) / res["graph"],
            "fwd_bwd": {"value": ss / res["fwdbwd"], "ms_per_call": 1e3 * res["fwdbwd"]},
            "plain_gpu_first_wave": {"fwd_ms": 1e3 * res["plain_fwd_wave"], "fwd_bwd_ms": 1e3 * res["plain_fwdbwd_wave"],
                                     "fused_fwd_ms": 1e3 * res["fwd_wave"],
                                     "speedup_fwd": res["plain_fwd_wave"] / res["fwd_wave"],
                                     "screen_steps": ss_w},
            "create_seconds": t_create, "tune_seconds": t_tune,
            "workload": f"{len(inst)} serving-mix instances (N 256-2048, lambda 532/1064/1550 nm, 5-20 screens, "
                        "log-uniform Cn2, 3 subharmonic levels, R=1), waves of 256"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported by this build "
              f"(realizations shard without communication, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2604_07248_amd import api, binding, prof_summary, workloads

    cpu_rec = oracle_fields = None
    if args.only == "all" and not args.no_cpu_baseline:
        # the oracle on the host cores first, while no process has touched the GPU
        cpu_rec, oracle_fields = cpu_baseline(workloads.headline(args.realizations), args.cpu_pairs)

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    binding.lib()
    fams = ["row_fwd", "row_bwd", "row_plain", "row_moments", "col", "synth", "sh", "evolve", "stats", "finalize",
            "copy", "sum"]

    if args.tune_cache and os.path.exists(args.tune_cache):
        api.tune_cache_load(args.tune_cache)
    w = workloads.headline(args.realizations)
    path = w.path
    plan = api.Plan(path)
    # launch configuration: measured (or cached) before any timed step
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
                         "screen_steps_per_step": ss_per_step, "launch_config": widths}}

    def fwd(i):
        plan.propagate(u0, seed=w.seed, t=i, out=u_out)  # moments taken inside

    if args.only in ("all", "fwd"):
        plan.bind_moments(moments)
        sec, ktab, dom = measure(torch, fwd, args.steps, args.warmup, binding, fams, path, "fwd")
        plan.bind_moments(None)
        result["value"] = ss_per_step / sec
        result["ms_per_step"] = 1e3 * sec
        result["kernels"] = ktab
        # whole-path effective bandwidth: every family's algorithmic bytes per step
        result["path_effective_GBps"] = sum(step_bytes(path, "fwd").values()) / sec / 1e9
        result["roofline"] = roofline(ktab, dom, prof_summary.load_traffic(os.path.join(ROOT, "profiles"), "fwd"),
                                      path, "fwd", sec)
        if oracle_fields is not None:
            # the error against the FP64 oracle of the same step (t = 0) on the
            # realizations of the oracle's timed sample
            got = plan.propagate(u0, seed=w.seed, t=0)[:oracle_fields.shape[0]].cpu().numpy()
            err = np.linalg.norm(got.astype(np.complex128) - oracle_fields) / np.linalg.norm(oracle_fields)
            result["oracle_rel_l2"] = {"value": float(err), "realizations": int(oracle_fields.shape[0]),
                                       "tolerance": 1e-4, "what": "received fields of the forward step at t=0"}

    if args.only in ("all", "fwd_as"):
        # the same forward step with the angular-spectrum transfer function (Sec. 2.1)
        pas = path.with_(tf_kind=workloads.TF_ANGULAR_SPECTRUM)
        plan_as = api.Plan(pas)
        plan_as.tune()
        plan_as.bind_moments(moments)

        def fwd_as(i):
            plan_as.propagate(u0, seed=w.seed, t=i, out=u_out)

        sec, ktab, dom = measure(torch, fwd_as, args.steps, args.warmup, binding, fams, pas, "fwd")
        result["fwd_angular_spectrum"] = {"value": ss_per_step / sec, "unit": "screen-steps/s",
                                          "ms_per_step": 1e3 * sec, "kernels": ktab, "dominant": dom}
        plan_as.close()

    if args.only in ("all", "fwdbwd"):
        # checkpoints at the screen planes that also keep the screens' column
        # halves, so the adjoint synthesises no screen again
        plan_ck = api.Plan(path, flags=binding.SCREEN_CHECKPOINTS)
        plan_ck.tune()
        ck = plan_ck.new_checkpoints()

        def fwdbwd(i):
            out, c = plan_ck.propagate(u0, seed=w.seed, t=i, out=u_out, checkpoints=ck)
            plan_ck.propagate_backward(out, c, seed=w.seed, t=i, shared_source=True)

        sec, ktab, dom = measure(torch, fwdbwd, args.steps, args.warmup, binding, fams, path, "fwdbwd")
        result["fwd_bwd"] = {"value": ss_per_step / sec, "unit": "screen-steps/s", "ms_per_step": 1e3 * sec,
                             "kernels": ktab, "dominant": dom,
                             "path_effective_GBps": sum(step_bytes(path, "fwdbwd").values()) / sec / 1e9,
                             "step_frac_hbm": sum(step_bytes(path, "fwdbwd").values()) / sec / 1e9 / HBM_PEAK_GBPS,
                             "checkpoint_bytes": ck.numel() * 8}
        del ck
        plan_ck.close()

    if args.only in ("all", "fwdbwd_rev"):
        # the checkpoint-free adjoint: screen-plane fields rebuilt from u_out
        def fwdbwd_rev(i):
            out = plan.propagate(u0, seed=w.seed, t=i, out=u_out)
            plan.propagate_backward(out, None, seed=w.seed, t=i, u_out=out, shared_source=True)

        sec, ktab, dom = measure(torch, fwdbwd_rev, args.steps, args.warmup, binding, fams, path, "fwdbwd_rev")
        ck_bytes = path.realizations * path.num_screens * path.n * path.n * 8
        result["fwd_bwd_reversible"] = {"value": ss_per_step / sec, "unit": "screen-steps/s",
                                        "ms_per_step": 1e3 * sec, "kernels": ktab, "dominant": dom,
                                        "checkpoint_bytes_saved": ck_bytes - 2 * path.realizations * path.n * path.n * 8,
                                        "step_frac_hbm": sum(step_bytes(path, "fwdbwd_rev").values()) / sec / 1e9
                                        / HBM_PEAK_GBPS}

    if args.only in ("all", "ar"):
        w3 = workloads.config3()
        p3 = w3.path
        plan3 = api.Plan(p3)
        plan3.tune()
        spec = plan3.init_spectra(w3.seed)
        u3 = torch.from_numpy(w3.source_field().astype(np.complex64)).to(dev)
        o3 = torch.empty((p3.realizations, p3.n, p3.n), dtype=torch.complex64, device=dev)
        m3 = api.Moments(p3.n, p3.dx)
        plan3.bind_moments(m3)  # the moments of every step, inside its final row pass
        ex = w3.extra

        def ar(i):
            # one AR time step: the evolution fused into the screen synthesis
            plan3.evolve_propagate(spec, w3.seed, i + 1, ex["alpha"], ex["shift_x"], ex["shift_y"], u_in=u3, out=o3)

        def ar_two_calls(i):
            plan3.evolve(spec, w3.seed, i + 1, ex["alpha"], ex["shift_x"], ex["shift_y"])
            plan3.propagate(u3, spectra=spec, out=o3)

        run_steps(torch, ar_two_calls, 0, 2)
        t0 = time.perf_counter()
        run_steps(torch, ar_two_calls, 2, args.steps)
        sec_two = (time.perf_counter() - t0) / args.steps
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
                        "two_calls_ms_per_step": 1e3 * sec_two, "launch_config": plan3.config,
                        "graph_seconds_for_1000_steps": 1000 * sec_graph,
                        "path_effective_GBps": sum(step_bytes(p3, "ar").values()) / sec / 1e9}
        plan3.close()
        del spec

    if args.only in ("all", "uneven"):
        result["uneven_batch"] = uneven_leg(torch, np, api, workloads, args, dev)

    if args.only in ("all", "plain"):
        # one op per kernel: screens from turpy_noise + torch ops, then Eq. 1
        # with torch.fft and elementwise ops; forward, and forward + backward
        # through torch's autograd (gradients of the shared source and of the
        # screens, as in the fused fwd_bwd leg)
        H = fresnel_tables(torch, np, path, dev)
        amp = torch.from_numpy(psd_amplitudes(np, path)).to(dev)
        phi = torch.empty((path.realizations, path.num_screens, path.n, path.n), dtype=torch.float32, device=dev)

        def plain(i):
            plain_screens(torch, api, path, w.seed, i, amp, phi)
            moments.add(plain_propagate(torch, path, u0, H, phi))

        def plain_fb(i):
            plain_screens(torch, api, path, w.seed, i, amp, phi)
            u_in = u0.detach().requires_grad_(True)
            ph = phi.detach().requires_grad_(True)
            out = plain_propagate(torch, path, u_in, H, ph)
            torch.autograd.backward(out, grad_tensors=out.detach())

        res = {}
        for name, fn in (("fwd", plain), ("fwdbwd", plain_fb)):
            k = max(2, args.steps // 5)
            run_steps(torch, fn, 0, 2)
            t0 = time.perf_counter()
            run_steps(torch, fn, 2, k)
            res[name] = (time.perf_counter() - t0) / k
        # same noise, same physics: the agreement of the two versions
        fused = plan.propagate(u0, seed=w.seed, t=0)
        ref = plain_propagate(torch, path, u0, H, plain_screens(torch, api, path, w.seed, 0, amp, phi))
        diff = float(torch.linalg.vector_norm(fused - ref) / torch.linalg.vector_norm(ref))
        result["plain_gpu"] = {"value": ss_per_step / res["fwd"], "unit": "screen-steps/s",
                               "ms_per_step": 1e3 * res["fwd"],
                               "fwd_bwd": {"value": ss_per_step / res["fwdbwd"], "ms_per_step": 1e3 * res["fwdbwd"]},
                               "kind": "one op per kernel: turpy_noise, torch elementwise, torch.fft; "
                                       "backward by torch autograd",
                               "rel_l2_vs_fused": diff}
        if "value" in result:
            result["speedup_vs_plain"] = result["value"] / result["plain_gpu"]["value"]
        if "fwd_bwd" in result:
            result["fwd_bwd"]["speedup_vs_plain"] = result["fwd_bwd"]["value"] / result["plain_gpu"]["fwd_bwd"]["value"]
        del phi, H, amp

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
    if cpu_rec is not None:
        result["cpu_baseline"] = cpu_rec

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
