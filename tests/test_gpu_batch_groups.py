"""Grouped launches of uneven batches: the instances of a batch that share
the grid size, the realization count and the transfer-function form (and
have every distance > 0) run each pass of the forward pass and of the adjoint
as one launch for all of them.  Every instance must still equal its own
plan's call with the instance key bit for bit: fields, checkpoints and
gradients, with screen counts that differ inside a group, beside instances
that cannot join one, through graph replays, and in every transfer-function
form."""
import numpy as np
import pytest
import torch

from paper_2604_07248_amd import binding as B
from paper_2604_07248_amd import workloads

from gpu_helpers import TOL, oracle_propagate, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_2604_07248_amd import api as _api
    return _api


def _p(n, m, r=1, sh=3, lam=1.064e-6, tf=0, cn2=1e-14):
    dx = 2e-3 if n >= 128 else 4e-3
    limit = n * dx * dx / lam
    length = min(0.8 * limit * max(m, 1), 3000.0)
    return workloads.uniform_path(n, n * dx, lam, length, m, cn2, 0.005, 20.0, sh, realizations=r).with_(tf_kind=tf)


def _evanescent(m, r=1):
    # dx = lambda/2: bins beyond kappa = k, the angular-spectrum form with its table
    lam, dx, n = 1e-6, 0.5e-6, 64
    dz = (4e-6,) + (7e-6,) * (m - 1) + (4e-6,)
    return workloads.Path(n=n, dx=dx, wavelength=lam, dz=dz, cn2dz=(2e-17,) * m,
                          tf_kind=workloads.TF_ANGULAR_SPECTRUM, realizations=r)


def mixed_paths():
    A = workloads.TF_ANGULAR_SPECTRUM
    return [
        _p(64, 3), _p(64, 6, sh=0), _p(64, 1), _p(64, 4, lam=1.55e-6), _p(64, 6),      # one group, M 1..6
        _p(128, 2, r=2, tf=A), _p(128, 5, r=2, tf=A, sh=0), _p(128, 3, r=2, tf=A),     # angular spectrum, R = 2
        _evanescent(2), _evanescent(3),                                               # the tabulated form
        _p(256, 2, r=3), _p(256, 4, r=3),                                              # R = 3, odd pairs
        _p(64, 3).with_(dz=(0.0,) + _p(64, 3).dz[1:]),                                 # no first distance: alone
        _p(64, 2, r=2),                                                                # a key of its own
        workloads.Path(n=64, dx=4e-3, wavelength=1e-6, dz=(1.0,), cn2dz=(), realizations=1),  # no screens
        _p(512, 2), _p(512, 3),
    ]


def _sources(paths, batch):
    srcs = []
    for i, p in enumerate(paths):
        u0 = workloads.gaussian_source(p.n, p.dx, p.n * p.dx / 8) if p.dx > 1e-5 else workloads.seeded_field((p.n, p.n), i)
        srcs.append(torch.from_numpy(np.ascontiguousarray(np.broadcast_to(u0, (p.realizations, p.n, p.n)),
                                                          dtype=np.complex64)).cuda())
    return srcs, batch.pack(srcs)


@pytest.mark.parametrize("with_ck", [False, True])
def test_groups_equal_single_plans(api, with_ck):
    paths = mixed_paths()
    say(f"[groups] {len(paths)} instances, checkpoints={with_ck}")
    batch = api.Batch(paths)
    srcs, u_in = _sources(paths, batch)
    res = batch.propagate(u_in, seed=11, t=3, checkpoints=with_ck)
    out, ck = (res if with_ck else (res, None))
    outs = batch.unpack(out)
    if with_ck:
        rng = np.random.default_rng(4)
        g = torch.from_numpy((rng.standard_normal(batch.total) + 1j * rng.standard_normal(batch.total))
                             .astype(np.complex64)).cuda()
        g_in, g_phi = batch.propagate_backward(g, ck, seed=11, t=3)
        gins, gs = batch.unpack(g_in), batch.unpack(g)
    for i, p in enumerate(paths):
        plan = api.Plan(p)
        s_i = api.Batch.instance_seed(11, i)
        if with_ck:
            o, c = plan.propagate(srcs[i], seed=s_i, t=3, checkpoints=True)
            off, size = batch.ck_offsets[i], p.realizations * p.num_screens * p.n * p.n
            assert torch.equal(ck[off:off + size].view_as(c), c), i
            gi, gp = plan.propagate_backward(gs[i].contiguous(), c, seed=s_i, t=3)
            assert torch.equal(gins[i], gi), ("grad_in", i)
            assert torch.equal(g_phi[off:off + size].view_as(gp), gp), ("grad_phi", i)
        else:
            o = plan.propagate(srcs[i], seed=s_i, t=3)
        assert torch.equal(outs[i], o), (i, p.n, p.num_screens)
        plan.close()
    if with_ck:
        # without grad_u_in each member's own adjoint runs: the same dL/dphi
        size = B.batch_workspace_size(batch.handle, B.OP_PROPAGATE_BACKWARD)
        ws = torch.empty(max(size, 256), dtype=torch.uint8, device="cuda")
        g_phi2 = torch.empty_like(g_phi)
        B.batch_propagate_backward(batch.handle, 11, 3, g.data_ptr(), ck.data_ptr(), None, g_phi2.data_ptr(),
                                   ws.data_ptr(), size, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(g_phi2, g_phi)
    batch.close()


def test_groups_follow_tuned_radix(api):
    """A batch tuned after creation: the groups launch the radix plans the
    instances' plans hold now, so the bits still match single plans tuned the
    same way."""
    paths = [_p(512, 2, r=4), _p(512, 3, r=4), _p(512, 1, r=4)]
    batch = api.Batch(paths)
    srcs, u_in = _sources(paths, batch)
    batch.tune()
    out = batch.unpack(batch.propagate(u_in, seed=2))
    for i, p in enumerate(paths):
        plan = api.Plan(p)
        plan.tune()  # the same cache entries as the batch's plans
        assert torch.equal(out[i], plan.propagate(srcs[i], seed=api.Batch.instance_seed(2, i))), i


def test_grouped_graph_replays(api):
    paths = mixed_paths()[:8]
    batch, eager = api.Batch(paths), api.Batch(paths)
    _, u_in = _sources(paths, batch)
    out = torch.empty_like(u_in)
    t_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    batch.bind_time(t_dev)
    batch.propagate(u_in, seed=5, t=0, out=out)  # workspace allocated before the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.propagate(u_in, seed=5, t=0, out=out)
    for t in (2, 7, 2, 0):
        t_dev.fill_(t)
        graph.replay()
        torch.cuda.synchronize()
        got = out.clone()
        want = eager.propagate(u_in, seed=5, t=t)
        torch.cuda.synchronize()
        assert torch.equal(got, want), t
    batch.bind_time(None)
    say("[groups] 4 graph replays equal the eager calls")


def test_grouped_mix_full_wave(api):
    """A full wave of the serving mix (256 instances, one realization each):
    sampled instances of every grid size against their own plans, and per
    grid size the instance with the fewest screens against the oracle."""
    mix = [w.path for w in workloads.uneven_batch()][:256]
    batch = api.Batch(mix)
    srcs, u_in = _sources(mix, batch)
    outs = batch.unpack(batch.propagate(u_in, seed=9, t=1))
    rng = np.random.default_rng(3)
    sample = sorted(set(rng.choice(len(mix), 12, replace=False).tolist()) | {0, len(mix) - 1})
    for i in sample:
        plan = api.Plan(mix[i])
        assert torch.equal(outs[i], plan.propagate(srcs[i], seed=api.Batch.instance_seed(9, i), t=1)), i
        plan.close()
    say(f"[groups] serving-mix wave: {len(sample)} sampled instances bitwise")
    # per grid size, the instance with the fewest screens against the oracle
    for n in sorted({p.n for p in mix}):
        i = min((k for k, p in enumerate(mix) if p.n == n), key=lambda k: mix[k].num_screens)
        ref, _ = oracle_propagate(mix[i], api.Batch.instance_seed(9, i), srcs[i].cpu().numpy(), t=1)
        e = rel_l2(outs[i].cpu().numpy(), ref)
        say(f"[groups] instance {i}: N={n} M={mix[i].num_screens} against the oracle {e:.2e}")
        assert e < TOL, (i, e)
