"""turpy_propagate_static: the forward split-step without a workspace
argument, for callers that cannot allocate (graph capture, serving loops);
its scratch is a fixed device array of the library.  Checked against
turpy_propagate through the C ABI, bit for bit (same kernels, same
arithmetic), on two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2604_07248_amd import binding as B
from paper_2604_07248_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L(gpu_lib):
    gpu_lib.turpy_propagate_static.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p,
                                               ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p]
    gpu_lib.turpy_propagate_static.restype = ctypes.c_int32
    return gpu_lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _run_both(L, path, seed, t, shared, checkpoints):
    plan = B.plan_create(path)
    try:
        n, r, m = path.n, path.realizations, path.num_screens
        rng = np.random.default_rng(seed)
        shape = (n, n) if shared else (r, n, n)
        u_in = torch.from_numpy((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)).cuda()
        stride = 0 if shared else n * n
        outs = []
        for static in (False, True):
            u_out = torch.full((r, n, n), float("nan"), dtype=torch.complex64, device="cuda")
            ck = torch.full((r, m, n, n), float("nan"), dtype=torch.complex64, device="cuda") if checkpoints else None
            if static:
                st = L.turpy_propagate_static(plan, seed, t, _p(u_in), stride, B.SCREENS_SYNTH, None, _p(u_out),
                                              _p(ck), _stream())
                B.check(st)
            else:
                size = B.workspace_size(plan, B.OP_PROPAGATE)
                ws = torch.empty(max(size, 256), dtype=torch.uint8, device="cuda")
                B.propagate(plan, seed, t, _p(u_in), stride, B.SCREENS_SYNTH, None, _p(u_out), _p(ck), _p(ws), size,
                            _stream())
            torch.cuda.synchronize()
            outs.append((u_out.cpu().numpy(), None if ck is None else ck.cpu().numpy()))
        return outs
    finally:
        B.plan_destroy(plan)


def test_static_equals_workspace_entry_point(L):
    """Two calls in a row: a larger plan (N = 512, R = 10, subharmonics,
    checkpoints), then a smaller one (N = 256, R = 3, shared source) that finds
    the first call's data left in the array."""
    big = workloads.uniform_path(512, 1.0, 1.55e-6, 2000.0, 4, 1e-14, 0.005, 20.0, 3, realizations=10)
    small = workloads.uniform_path(256, 0.5, 1.55e-6, 1000.0, 3, 5e-15, 0.005, 20.0, 0, realizations=3)
    for path, shared, ck in ((big, False, True), (small, True, False)):
        (a, ca), (b, cb) = _run_both(L, path, seed=12, t=3, shared=shared, checkpoints=ck)
        assert np.isfinite(b).all()
        assert np.array_equal(a, b)
        if ck:
            assert np.array_equal(ca, cb)


def test_static_rejects_plans_beyond_the_array(L):
    """N = 1024 with 64 realizations needs 33 scratch planes (264 MiB), beyond
    the 64 MiB array: refused before anything is enqueued."""
    path = workloads.headline(64).path
    plan = B.plan_create(path)
    try:
        n = path.n
        u_in = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
        u_out = torch.zeros((64, n, n), dtype=torch.complex64, device="cuda")
        st = L.turpy_propagate_static(plan, 1, 0, _p(u_in), 0, B.SCREENS_SYNTH, None, _p(u_out), None, _stream())
        assert st == B.E_WORKSPACE and "static array" in B.last_error()
    finally:
        B.plan_destroy(plan)
