"""GPU parity of the dual-domain receiver and its adjoint against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import receiver as orx
from paper_2604_07248_amd import workloads

from gpu_helpers import TOL, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_2604_07248_amd import api as _api
    return _api


@pytest.mark.parametrize("n,batch", [(64, 3), (512, 5), (1024, 2)])
def test_receiver_forward_and_adjoint(api, n, batch):
    dx = 0.6 / n
    rng = np.random.default_rng(n)
    u = (workloads.gaussian_source(n, dx, 0.1)[None] *
         np.exp(1j * rng.standard_normal((batch, n, n)))).astype(np.complex64)
    t1 = (0.5 * rng.standard_normal((n, n))).astype(np.float32)
    t2 = (0.5 * rng.standard_normal((n, n))).astype(np.float32)
    g = (rng.standard_normal((batch, n, n)) + 1j * rng.standard_normal((batch, n, n))).astype(np.complex64)
    rx = api.Receiver(n, dx)
    cu = torch.from_numpy(u).cuda()
    c1, c2 = torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda()
    out = rx.forward(cu, c1, c2).cpu().numpy()
    ref = orx.forward(u.astype(np.complex128), t1.astype(np.float64), t2.astype(np.float64), dx)
    e = rel_l2(out, ref)
    g_u, d1, d2 = rx.backward(cu, c1, c2, torch.from_numpy(g).cuda())
    rg, r1, r2 = orx.adjoint(g.astype(np.complex128), u.astype(np.complex128), t1.astype(np.float64),
                             t2.astype(np.float64), dx)
    eg, e1, e2 = rel_l2(g_u.cpu().numpy(), rg), rel_l2(d1.cpu().numpy(), r1), rel_l2(d2.cpu().numpy(), r2)
    say(f"[receiver] n={n} batch={batch} out {e:.2e} grad_u {eg:.2e} dtheta1 {e1:.2e} dtheta2 {e2:.2e}")
    assert e < TOL and eg < TOL and e1 < TOL and e2 < TOL
    # determinism of the batch sums
    _, d1b, d2b = rx.backward(cu, c1, c2, torch.from_numpy(g).cuda())
    assert torch.equal(d1, d1b) and torch.equal(d2, d2b)


def test_zero_masks_identity(api):
    n, dx = 256, 0.002
    rng = np.random.default_rng(1)
    u = (rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))).astype(np.complex64)
    rx = api.Receiver(n, dx)
    z = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    out = rx.forward(torch.from_numpy(u).cuda(), z, z).cpu().numpy()
    ref = orx.aperture(n, dx) * u
    assert rel_l2(out, ref) < 1e-5
