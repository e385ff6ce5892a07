"""Dual-domain two-mask receiver and its adjoint, FP64 (Sec. 2.5, Sec. 4.1).

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

The received field is apodised by a circular aperture (12 inch = 0.3048 m
diameter), multiplied by a learnable real-space phase mask theta1, carried to
the Fourier plane by a lens (a DFT), multiplied by a learnable Fourier-plane
mask theta2, and carried back by a second lens (an inverse DFT):
  U1 = A U exp(i theta1);  Z = DFT{U1} exp(i theta2');  U_out = IDFT{Z}
theta2 is stored in centred (fftshift) order: theta2' = ifftshift(theta2).
The unitary lens pair is equivalent to the unnormalised DFT / 1/N^2 inverse
pair used here.  Adjoint (g = dL/dRe + i dL/dIm):
  g_Z = DFT{g_out} / N^2;  dL/dtheta2' = sum_b Im(conj(Z) g_Z);
  g_U1 = IDFT{conj(exp(i theta2')) DFT{g_out}};  dL/dtheta1 = sum_b Im(conj(U1) g_U1);
  g_U = A exp(-i theta1) g_U1.
"""

import numpy as np

APERTURE_DIAMETER = 0.3048


def aperture(n, dx, diameter=APERTURE_DIAMETER):
    x = (np.arange(n) - n // 2) * dx
    return ((x[None, :] ** 2 + x[:, None] ** 2) <= (0.5 * diameter) ** 2).astype(np.float64)


def forward(u, theta1, theta2, dx, diameter=APERTURE_DIAMETER):
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[-1]
    u1 = aperture(n, dx, diameter) * u * np.exp(1j * theta1)
    z = np.fft.fft2(u1) * np.exp(1j * np.fft.ifftshift(theta2))
    return np.fft.ifft2(z)


def adjoint(g_out, u, theta1, theta2, dx, diameter=APERTURE_DIAMETER):
    """Returns (g_u [B][N][N], dtheta1 [N][N], dtheta2 [N][N] centred order)."""
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[-1]
    a = aperture(n, dx, diameter)
    u1 = a * u * np.exp(1j * theta1)
    m2 = np.exp(1j * np.fft.ifftshift(theta2))
    z = np.fft.fft2(u1) * m2
    gf = np.fft.fft2(np.asarray(g_out, dtype=np.complex128))
    g_z = gf / (n * n)
    dth2 = np.imag(np.conj(z) * g_z).reshape(-1, n, n).sum(axis=0)
    g_u1 = np.fft.ifft2(np.conj(m2) * gf)
    dth1 = np.imag(np.conj(u1) * g_u1).reshape(-1, n, n).sum(axis=0)
    g_u = a * np.exp(-1j * theta1) * g_u1
    return g_u, dth1, np.fft.fftshift(dth2)
