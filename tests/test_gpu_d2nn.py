"""Differentiable training path (fp32 masks, complex64 fields): N=512, 6 weak
screens, two 512x512 masks behind the path.  GPU gradients of the training
loss against the FP64 oracle's adjoint (full masks, full batch of 64) and
against FP64 central differences on 8x8 mask subsets; the path adjoint is
exercised through dL/du_in and dL/dphi as well."""
import numpy as np
import pytest
import torch

from oracle import propagate as opr
from oracle import receiver as orx
from paper_2604_07248_amd import workloads

from gpu_helpers import TOL, oracle_screens, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods(gpu_lib):
    from paper_2604_07248_amd import api, d2nn
    return api, d2nn


def np_loss_and_grad(u_out, i_vac, ap):
    """The training loss in float64 and its gradient dL/dRe + i dL/dIm."""
    inten = np.abs(u_out) ** 2
    b = inten.shape[0]
    m1 = inten.mean(0)
    var = ((inten - m1) ** 2).mean(0)
    num, den = np.sum(var * ap), np.sum(m1 * m1 * ap)
    d2 = np.sum(i_vac ** 2)
    loss = num / den + np.sum((m1 - i_vac) ** 2) / d2
    # dL/dI[b, x]
    d_var = ap / den
    d_m1 = -num / den ** 2 * 2 * m1 * ap + 2 * (m1 - i_vac) / d2
    d_i = d_var * 2 * (inten - m1) / b + d_m1 / b
    return loss, 2 * d_i * u_out


def test_training_gradients_match_oracle(mods):
    api, d2nn = mods
    w = workloads.config4()
    p = w.path
    say("[d2nn] N=512 batch=64 M=6")
    tr = d2nn.D2NNTrainer(w, epochs=10)
    rng = np.random.default_rng(5)
    with torch.no_grad():  # non-trivial masks so that every factor of the adjoint matters
        tr.theta1.copy_(torch.from_numpy((0.3 * rng.standard_normal((p.n, p.n))).astype(np.float32)))
        tr.theta2.copy_(torch.from_numpy((0.3 * rng.standard_normal((p.n, p.n))).astype(np.float32)))
    epoch = 3
    u_out = tr.forward(epoch)
    loss = d2nn.loss_fn(u_out, tr.i_vac, tr.aperture)
    loss.backward()
    g1, g2 = tr.theta1.grad.cpu().numpy(), tr.theta2.grad.cpu().numpy()
    # oracle: same screens (seed, t = epoch), float64 throughout
    t1 = tr.theta1.detach().cpu().numpy().astype(np.float64)
    t2 = tr.theta2.detach().cpu().numpy().astype(np.float64)
    u0 = w.source_field().astype(np.complex64).astype(np.complex128)
    phi = oracle_screens(p, w.seed, range(p.realizations), t=epoch)
    u_rx, _ = opr.propagate(u0, p, phi)
    vac, _ = opr.propagate(u0, p, np.zeros((1,) + phi.shape[1:]))
    zero = np.zeros((p.n, p.n))
    i_vac = np.abs(orx.forward(vac, zero, zero, p.dx)[0]) ** 2
    ap = orx.aperture(p.n, p.dx)
    out = orx.forward(u_rx, t1, t2, p.dx)
    ref_loss, g_out = np_loss_and_grad(out, i_vac, ap)
    _, r1, r2 = orx.adjoint(g_out, u_rx, t1, t2, p.dx)
    e_loss = abs(float(loss) - ref_loss) / abs(ref_loss)
    e1, e2 = rel_l2(g1, r1), rel_l2(g2, r2)
    say(f"[d2nn] loss {float(loss):.6f} vs {ref_loss:.6f} ({e_loss:.1e}); dtheta1 {e1:.2e} dtheta2 {e2:.2e}")
    # the mask gradients to the adjoint bound of every other test (measured: a few 1e-6)
    assert e_loss < TOL and e1 < TOL and e2 < TOL

    # central differences (FP64 oracle) on central 8x8 subsets, 4 realizations
    sub = slice(p.n // 2 - 4, p.n // 2 + 4)
    ur4 = u_rx[:4]
    out4 = orx.forward(ur4, t1, t2, p.dx)
    _, g4 = np_loss_and_grad(out4, i_vac, ap)
    _, a1, a2 = orx.adjoint(g4, ur4, t1, t2, p.dx)
    u4 = torch.from_numpy(ur4.astype(np.complex64)).cuda()
    th1, th2 = tr.theta1.detach().clone().requires_grad_(), tr.theta2.detach().clone().requires_grad_()
    l4 = d2nn.loss_fn(api.ReceiverFn.apply(u4, th1, th2, tr.rx), tr.i_vac, tr.aperture)
    l4.backward()
    gpu1, gpu2 = th1.grad.cpu().numpy()[sub, sub], th2.grad.cpu().numpy()[sub, sub]
    h = 1e-5
    fd1, fd2 = np.zeros((8, 8)), np.zeros((8, 8))
    for i in range(8):
        for j in range(8):
            for t, fd in ((0, fd1), (1, fd2)):
                e = np.zeros((p.n, p.n))
                e[p.n // 2 - 4 + i, p.n // 2 - 4 + j] = h
                a, b = (t1 + e, t2) if t == 0 else (t1, t2 + e)
                c, d = (t1 - e, t2) if t == 0 else (t1, t2 - e)
                lp, _ = np_loss_and_grad(orx.forward(ur4, a, b, p.dx), i_vac, ap)
                lm, _ = np_loss_and_grad(orx.forward(ur4, c, d, p.dx), i_vac, ap)
                fd[i, j] = (lp - lm) / (2 * h)
    s1, s2 = np.abs(fd1).max(), np.abs(fd2).max()
    say(f"[d2nn] FD 8x8: oracle adjoint {np.abs(a1[sub, sub] - fd1).max() / s1:.1e}/"
        f"{np.abs(a2[sub, sub] - fd2).max() / s2:.1e}, GPU {np.abs(gpu1 - fd1).max() / s1:.1e}/"
        f"{np.abs(gpu2 - fd2).max() / s2:.1e}")
    assert np.abs(a1[sub, sub] - fd1).max() < 1e-6 * s1 and np.abs(a2[sub, sub] - fd2).max() < 1e-6 * s2
    assert np.abs(gpu1 - fd1).max() < 2e-3 * s1 and np.abs(gpu2 - fd2).max() < 2e-3 * s2


def test_path_adjoint_through_autograd(mods):
    """dL/du_in and dL/dphi through Propagate.apply against the oracle adjoint."""
    api, _ = mods
    w = workloads.config4(batch=4)
    p = w.path
    plan = api.Plan(p)
    u0 = torch.from_numpy(w.source_field().astype(np.complex64)).cuda().requires_grad_()
    phi = plan.screens(seed=w.seed).requires_grad_()
    out = api.Propagate.apply(u0, phi, plan, 0, 0)
    weight = torch.linspace(0.5, 1.5, p.n, device="cuda")[None, :]
    loss = ((out.real ** 2 + out.imag ** 2) * weight).sum()
    loss.backward()
    phi64 = oracle_screens(p, w.seed, range(p.realizations))
    ref, ck = opr.propagate(w.source_field().astype(np.complex64).astype(np.complex128), p, phi64)
    g = 2 * weight.cpu().numpy().astype(np.float64) * ref
    g_in, g_phi = opr.propagate_adjoint(g, p, phi64, ck)
    e_in, e_phi = rel_l2(u0.grad.cpu().numpy(), g_in.sum(0)), rel_l2(phi.grad.cpu().numpy(), g_phi)
    say(f"[autograd] grad u_in {e_in:.2e} grad phi {e_phi:.2e}")
    assert e_in < TOL and e_phi < TOL


def test_training_reduces_loss(mods):
    api, d2nn = mods
    w = workloads.config4(batch=16)
    tr = d2nn.D2NNTrainer(w, lr=0.05, epochs=30)
    losses = [float(tr.step(e)) for e in range(30)]
    say(f"[d2nn] loss {losses[0]:.4f} -> {np.mean(losses[-5:]):.4f}")
    assert np.mean(losses[-5:]) < losses[0]
