"""Calls of every kernel family on small seeded inputs, for the LDS-poison
check: tests/test_gpu_lds_poison.py runs them in-process with the product
library and in a child process with the poison build (TURPY_LIBRARY), and
compares the outputs.  Run as a script: python lds_poison_cases.py OUT.npz."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _path(workloads, n, m, r, sh=0, tf=0):
    lam = 1e-6
    dx = 2e-3 if n >= 128 else 4e-3
    limit = n * dx * dx / lam
    return workloads.uniform_path(n, n * dx, lam, min(0.8 * limit * max(m, 1), 2000.0), m, 1e-14, 0.005, 20.0, sh,
                                  realizations=r).with_(tf_kind=tf)


def run_cases():
    """{name: numpy array} of every output."""
    import torch

    from paper_2604_07248_amd import api, binding, workloads
    binding.lib()
    out = {}

    def keep(name, t):
        torch.cuda.synchronize()
        out[name] = t.detach().cpu().numpy().copy()

    def c64(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()

    # forward, adjoint and screens at every row-pass schedule: row_pass (N <= 32),
    # pair (checkpoints), relay (N <= 1024), pair at N = 2048
    for n, r, sh, tf in ((16, 3, 0, 0), (64, 3, 3, 1), (256, 4, 3, 0), (1024, 2, 0, 0), (2048, 2, 3, 0)):
        p = _path(workloads, n, 2, r, sh, tf)
        plan = api.Plan(p)
        u0 = c64(workloads.gaussian_source(n, p.dx, 0.1 * n * p.dx))
        keep(f"fwd{n}", plan.propagate(u0, seed=5))
        o, ck = plan.propagate(u0, seed=5, checkpoints=True)
        keep(f"fwd_ck{n}", o)
        g_in, g_phi = plan.propagate_backward(o, ck, seed=5)
        keep(f"grad_in{n}", g_in)
        keep(f"grad_phi{n}", g_phi)
        keep(f"screens{n}", plan.screens(seed=5))
        m = api.Moments(n, p.dx)
        plan.bind_moments(m)
        plan.propagate(u0, seed=6)
        keep(f"moments{n}", m.buf)
        si, summary = m.finalize(power_fraction=0.99)
        keep(f"si{n}", si)
        out[f"summary{n}"] = np.array([summary[k] for k in ("si_plane", "w_2nd", "w_fit", "si_sum")])
        plan.close()
    # AR step fused into the synthesis
    p = _path(workloads, 256, 3, 4, 3)
    plan = api.Plan(p)
    spec = plan.init_spectra(7)
    u0 = c64(workloads.gaussian_source(256, p.dx, 0.1 * 256 * p.dx))
    keep("ar", plan.evolve_propagate(spec, 7, 1, 0.95, 0.3, -0.2, u_in=u0))
    keep("ar_state", spec)
    # receiver forward and adjoint
    n = 128
    rec = api.Receiver(n, 2e-3)
    rng = np.random.default_rng(4)
    u = c64(rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n)))
    th1 = torch.from_numpy(rng.uniform(-3, 3, (n, n)).astype(np.float32)).cuda()
    th2 = torch.from_numpy(rng.uniform(-3, 3, (n, n)).astype(np.float32)).cuda()
    y = rec.forward(u, th1, th2)
    keep("recv", y)
    gu, g1, g2 = rec.backward(u, th1, th2, y)
    keep("recv_gu", gu)
    keep("recv_g1", g1)
    keep("recv_g2", g2)
    # an uneven batch with groups
    paths = [_path(workloads, 64, m, 1, 3) for m in (1, 3, 2)] + [_path(workloads, 128, 2, 2)]
    batch = api.Batch(paths)
    src = batch.pack([torch.from_numpy(workloads.gaussian_source(q.n, q.dx, 0.1 * q.n * q.dx).astype(np.complex64))
                      .expand(q.realizations, q.n, q.n) for q in paths])
    bo, bck = batch.propagate(src, seed=3, checkpoints=True)
    keep("batch", bo)
    bg, bphi = batch.propagate_backward(bo, bck, seed=3)
    keep("batch_grad", bg)
    keep("batch_phi", bphi)
    return out


if __name__ == "__main__":
    res = run_cases()
    np.savez(sys.argv[1], **res)
