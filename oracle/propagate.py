"""Split-step propagation and its adjoint, FP64 (Sec. 2.1 Eq. 1, Sec. 2.4).

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

Eq. 1: U <- IDFT{ DFT{U} . H(dz) } . exp(i phi).  The path is described by
dz[0..M] (diffraction distance before screen i, and after the last screen) and
one screen per interval.  A zero distance skips the diffraction.  The constant
exp(i k dz) piston of the transfer function is dropped.

Transfer functions (frequencies f in cycles/m, df = 1/(N dx)):
  Fresnel:            H = exp(-i pi (lambda/n0) dz (fx^2 + fy^2))
  angular spectrum:   H = exp(i dz (sqrt(k^2 - kappa^2) - k)), kappa = 2 pi f,
                      k = 2 pi n0/lambda (Sec. 2.4); the phase is evaluated as
                      -dz kappa^2 / (sqrt(k^2 - kappa^2) + k) to avoid
                      cancellation; beyond kappa = k the wave is evanescent,
                      |H| = exp(-dz sqrt(kappa^2 - k^2)).
Adjoint (gradient convention g = dL/dRe U + i dL/dIm U, as PyTorch uses):
  through the diffraction: g <- IDFT{ conj(H) . DFT{g} } (P is unitary);
  through the screen: dL/dphi = Im(conj(W) g) with W the field just after the
  screen, then g <- exp(-i phi) g.
"""

import numpy as np

from .screens import signed_bins

TF_FRESNEL = 0
TF_ANGULAR_SPECTRUM = 1


def transfer_function(n, dx, wavelength, n0, dz, kind=TF_FRESNEL):
    df = 1.0 / (n * dx)
    kh = signed_bins(n)
    f2 = (kh[:, None] ** 2 + kh[None, :] ** 2) * df * df
    if kind == TF_FRESNEL:
        return np.exp(-1j * np.pi * (wavelength / n0) * dz * f2)
    k = 2.0 * np.pi * n0 / wavelength
    kap2 = 4.0 * np.pi ** 2 * f2
    prop = kap2 < k * k
    h = np.empty_like(f2, dtype=np.complex128)
    s = np.sqrt(np.where(prop, k * k - kap2, 0.0))
    h[prop] = np.exp(1j * (-dz * kap2[prop] / (s[prop] + k)))
    ev = ~prop
    h[ev] = np.exp(-dz * np.sqrt(kap2[ev] - k * k)) * np.exp(-1j * k * dz)
    return h


def diffract(u, h):
    """Eq. 1, first factor: IDFT{DFT{U} H} over the last two axes."""
    return np.fft.ifft2(np.fft.fft2(u) * h)


def diffract_adjoint(g, h):
    return np.fft.ifft2(np.fft.fft2(g) * np.conj(h))


def _tf(path, dz):
    return transfer_function(int(path.n), path.dx, path.wavelength, path.n0, dz,
                             int(getattr(path, "tf_kind", TF_FRESNEL)))


def propagate(u0, path, screens):
    """Forward split-step.

    u0:      complex [N][N] (shared source) or [R][N][N].
    screens: real [R][M][N][N] in radians.
    Returns (u_out [R][N][N], checkpoints [R][M][N][N]) where checkpoint i is the
    field right after screen i.
    """
    screens = np.asarray(screens, dtype=np.float64)
    r, m = screens.shape[0], screens.shape[1]
    u = np.broadcast_to(np.asarray(u0, dtype=np.complex128), (r,) + screens.shape[2:]).copy()
    ckpt = np.empty(screens.shape, dtype=np.complex128)
    for i in range(m):
        if path.dz[i] > 0:
            u = diffract(u, _tf(path, path.dz[i]))
        u = u * np.exp(1j * screens[:, i])
        ckpt[:, i] = u
    if path.dz[m] > 0:
        u = diffract(u, _tf(path, path.dz[m]))
    return u, ckpt


def propagate_adjoint(g_out, path, screens, checkpoints):
    """Adjoint of propagate(): returns (dL/du_in [R][N][N], dL/dphi [R][M][N][N])."""
    screens = np.asarray(screens, dtype=np.float64)
    m = screens.shape[1]
    g = np.array(g_out, dtype=np.complex128)
    gphi = np.empty(screens.shape, dtype=np.float64)
    if path.dz[m] > 0:
        g = diffract_adjoint(g, _tf(path, path.dz[m]))
    for i in range(m - 1, -1, -1):
        gphi[:, i] = np.imag(np.conj(checkpoints[:, i]) * g)
        g = g * np.exp(-1j * screens[:, i])
        if path.dz[i] > 0:
            g = diffract_adjoint(g, _tf(path, path.dz[i]))
    return g, gphi
