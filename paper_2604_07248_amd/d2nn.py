"""Training a dual-domain two-mask receiver through turbulence (Sec. 2.5, Sec. 4).

Each epoch propagates a batch through fresh screens (time index = epoch) with
the fused GPU path, applies the receiver with the two learnable masks, and
minimises scintillation inside the aperture plus the L2 distance of the mean
intensity to the vacuum beam through the same receiver:

    L = sum_A Var_b(I) / sum_A (E_b I)^2 + sum (E_b I - I_vac)^2 / sum I_vac^2

with Adam and a one-cycle learning-rate schedule from a constant (zero) phase
initialisation (Sec. 2.5).  The loss is a handful of reductions over |U|^2 in
PyTorch; propagation and receiver (forward and adjoint) run in libturpy.
"""

import numpy as np
import torch

from . import api


def loss_fn(u_out, i_vac, aperture):
    inten = u_out.real ** 2 + u_out.imag ** 2
    m1 = inten.mean(0)
    var = ((inten - m1) ** 2).mean(0)
    l_si = (var * aperture).sum() / ((m1 * m1) * aperture).sum()
    l_l2 = ((m1 - i_vac) ** 2).sum() / (i_vac * i_vac).sum()
    return l_si + l_l2


def aperture_mask(n, dx, diameter, device):
    x = (torch.arange(n, dtype=torch.float64, device=device) - n // 2) * dx
    return ((x[None, :] ** 2 + x[:, None] ** 2) <= (0.5 * diameter) ** 2).to(torch.float32)


class D2NNTrainer:
    def __init__(self, workload, diameter=0.3048, lr=0.01, epochs=100, device="cuda"):
        p = workload.path
        self.w, self.path = workload, p
        self.plan = api.Plan(p)
        self.rx = api.Receiver(p.n, p.dx, diameter)
        self.u0 = torch.from_numpy(workload.source_field().astype(np.complex64)).to(device)
        vac = api.Plan(p.with_(cn2dz=tuple(0.0 for _ in p.cn2dz), realizations=1))
        zero = torch.zeros((p.n, p.n), dtype=torch.float32, device=device)
        u_vac = self.rx.forward(vac.propagate(self.u0), zero, zero)
        self.i_vac = (u_vac.real ** 2 + u_vac.imag ** 2)[0]
        vac.close()
        self.aperture = aperture_mask(p.n, p.dx, diameter, device)
        self.theta1 = torch.zeros((p.n, p.n), dtype=torch.float32, device=device, requires_grad=True)
        self.theta2 = torch.zeros((p.n, p.n), dtype=torch.float32, device=device, requires_grad=True)
        self.opt = torch.optim.Adam([self.theta1, self.theta2], lr=lr)
        self.sched = torch.optim.lr_scheduler.OneCycleLR(self.opt, max_lr=lr, total_steps=epochs)

    def forward(self, epoch):
        u_rx = api.Propagate.apply(self.u0, None, self.plan, self.w.seed, epoch)
        return api.ReceiverFn.apply(u_rx, self.theta1, self.theta2, self.rx)

    def step(self, epoch):
        self.opt.zero_grad(set_to_none=True)
        loss = loss_fn(self.forward(epoch), self.i_vac, self.aperture)
        loss.backward()
        self.opt.step()
        self.sched.step()
        return loss.detach()
