"""Error handling forced from the host, with every kernel exiting normally:
the output check of TURPY_CHECK_FINITE plans, and kernel launches made to
fail by turpy_debug_fail_launch, after which plans and batches must give the
same bits as before."""
import numpy as np
import pytest
import torch

from paper_2604_07248_amd import binding as B
from paper_2604_07248_amd import workloads

from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_2604_07248_amd import api as _api
    return _api


@pytest.fixture(autouse=True)
def disarm(gpu_lib):
    yield
    B.debug_fail_launch(0)


def _path(n=64, r=3, m=3, sh=3):
    lam, dx = 1e-6, 4e-3
    limit = n * dx * dx / lam
    return workloads.uniform_path(n, n * dx, lam, 0.8 * limit * m, m, 1e-15, 0.005, 20.0, sh, realizations=r)


def _source(path):
    u0 = workloads.gaussian_source(path.n, path.dx, 0.1 * path.n * path.dx)
    return torch.from_numpy(np.ascontiguousarray(u0, dtype=np.complex64)).cuda()


def test_check_finite_clean_outputs_unchanged(api):
    path = _path()
    checked, plain = api.Plan(path, flags=B.CHECK_FINITE), api.Plan(path)
    u = _source(path)
    a, ca = checked.propagate(u, seed=1, checkpoints=True)
    b, cb = plain.propagate(u, seed=1, checkpoints=True)
    assert torch.equal(a, b) and torch.equal(ca, cb)
    ga = checked.propagate_backward(b, cb, seed=1, shared_source=True)
    gb = plain.propagate_backward(b, cb, seed=1, shared_source=True)
    assert torch.equal(ga[0], gb[0]) and torch.equal(ga[1], gb[1])
    assert torch.equal(checked.screens(seed=1), plain.screens(seed=1))


def test_check_finite_names_the_output(api):
    path = _path()
    checked = api.Plan(path, flags=B.CHECK_FINITE)
    u = _source(path).expand(path.realizations, path.n, path.n).clone()
    u[1, 5, 7] = complex(float("nan"), 0.0)
    with pytest.raises(B.TurpyError) as e:
        checked.propagate(u, seed=1)
    assert e.value.status == B.E_NONFINITE and "u_out" in str(e.value)
    out, ck = checked.propagate(_source(path), seed=1, checkpoints=True)
    g = out.clone()
    g[0, 3, 3] = complex(float("inf"), 0.0)
    with pytest.raises(B.TurpyError) as e:
        checked.propagate_backward(g, ck, seed=1)
    assert e.value.status == B.E_NONFINITE and "grad_u_in" in str(e.value)
    say(f"[finite] {e.value}")


def test_check_finite_refuses_capture(api):
    path = _path()
    checked = api.Plan(path, flags=B.CHECK_FINITE)
    u = _source(path)
    out = checked.propagate(u, seed=1)  # workspace allocated outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(graph):
        try:
            checked.propagate(u, seed=1, out=out)  # refused before anything is enqueued
        except B.TurpyError as e:
            err = e
    del graph
    assert err is not None and err.status == B.E_INVALID and "capturing" in str(err)


def test_release_during_capture_is_deferred(api):
    """A plan or batch released inside a graph capture (as the garbage
    collector may do) is destroyed after the capture: destroying it frees
    device memory, which would invalidate the capture."""
    path = _path()
    plan, batch = api.Plan(path), api.Batch([path, _path(n=128)])
    handles = (plan.handle, batch.handle)
    x = torch.zeros(8, device="cuda")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        x.add_(1.0)
        plan.close()
        batch.close()
        pending = [h for _, h in api._deferred]
        assert all(any(h is p for p in pending) for h in handles)
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    assert float(x.sum()) == 8 * 3
    api.Plan(path).close()  # a new plan destroys the deferred handles first
    assert not api._deferred
    del graph


def _sweep(call, check, limit=400):
    """Fail launch k of `call` for k = 1, 2, ... until a call enqueues fewer
    than k launches; after each failure `check` must see correct results.
    Returns the number of launches of one call."""
    for k in range(1, limit):
        B.debug_fail_launch(k)
        try:
            call()
            B.debug_fail_launch(0)
            return k - 1
        except B.TurpyError as e:
            assert e.status == B.E_HIP and "injected" in str(e), str(e)
        B.debug_fail_launch(0)
        check()
    raise AssertionError("the call never completed")


def test_injected_failures_forward_and_adjoint(api):
    path = _path()
    plan = api.Plan(path)
    u = _source(path)
    ref, ref_ck = plan.propagate(u, seed=2, checkpoints=True)
    ref_g = plan.propagate_backward(ref, ref_ck, seed=2, shared_source=True)
    torch.cuda.synchronize()

    def check():
        o, c = plan.propagate(u, seed=2, checkpoints=True)
        g = plan.propagate_backward(o, c, seed=2, shared_source=True)
        assert torch.equal(o, ref) and torch.equal(c, ref_ck)
        assert torch.equal(g[0], ref_g[0]) and torch.equal(g[1], ref_g[1])

    fwd = _sweep(lambda: plan.propagate(u, seed=2, checkpoints=True), check)
    bwd = _sweep(lambda: plan.propagate_backward(ref, ref_ck, seed=2, shared_source=True), check)
    say(f"[inject] forward {fwd} launches, adjoint {bwd}")
    assert fwd >= 2 * path.num_screens and bwd >= 2 * path.num_screens


def test_injected_failures_ar_step(api):
    path = _path(r=4)
    plan = api.Plan(path)
    u = _source(path)
    state = plan.init_spectra(3)
    raw = torch.empty(0, dtype=torch.uint8, device=state.device).set_(state.untyped_storage())  # the whole state
    keep = raw.clone()
    ref = plan.evolve_propagate(state, 3, 1, 0.9, 0.25, 0.5, u_in=u).clone()
    ref_state = raw.clone()

    def call():
        raw.copy_(keep)
        return plan.evolve_propagate(state, 3, 1, 0.9, 0.25, 0.5, u_in=u)

    def check():
        assert torch.equal(call(), ref) and torch.equal(raw, ref_state)

    k = _sweep(call, check)
    say(f"[inject] AR step {k} launches")
    assert k >= path.num_screens


def test_injected_failures_batch(api):
    paths = [_path(n=64, r=1, m=3), _path(n=128, r=2, m=2), _path(n=64, r=1, m=4), _path(n=32, r=3, m=1)]
    batch = api.Batch(paths)
    fields = [_source(p).cpu()[None].expand(p.realizations, p.n, p.n) for p in paths]
    src = batch.pack(fields)
    ref = batch.propagate(src, seed=4).clone()
    torch.cuda.synchronize()

    def check():
        assert torch.equal(batch.propagate(src, seed=4), ref)

    k = _sweep(lambda: batch.propagate(src, seed=4), check)
    say(f"[inject] batch {k} launches")
    assert k >= len(paths) * 3
