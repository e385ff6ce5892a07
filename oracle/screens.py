"""Phase-screen synthesis, FP64 (App. B Eq. S16, App. C Eq. S17-S18, Sec. 2.2
Eq. 2-3).

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

Conventions (readings of the paper, listed in the design notes):
  * arrays A[i0][i1], i0 <-> y, i1 <-> x; signed bin k^ = k for k < N/2 else k - N;
    f_k = k^ * df with df = 1/(N dx) in cycles per metre (Sec. 2.4 states the
    k-space step as 1/(N dx)).
  * Eq. S17 is evaluated with frequencies in cycles/m: W(f) = 0.023 r0^(-5/3)
    exp(-f^2/fm^2) / (f^2 + f0^2)^(11/6), fm = 1/l0 (kappa_m = 2 pi/l0 written
    in cycles/m), f0 = 1/L0.  This is the reading under which the 0.023 constant
    yields the Kolmogorov structure function 6.88 (r/r0)^(5/3).
  * Eq. S16: c[k] = N_c[k] sqrt(W(f_k)) df with c[0][0] = 0, and the screen is
    the inverse DFT without the 1/N^2 factor: z = sum_k c[k] exp(+2 pi i k.x/N).
  * One complex z serves two realizations: Re z for realization 2j, Im z for
    2j+1 (independent, identically distributed screens because W is even).
  * Eq. 2 (Lane subharmonics) with scale s = 3: level p uses df_p = df/3^p and
    the 8 non-centre points of the 3x3 grid; coordinates x = (i1 - N/2) dx,
    y = (i0 - N/2) dx.  Eq. 3 adds it to the main screen, and the mean of the
    result is removed (piston, App. B after Eq. S16).
"""

import numpy as np

from .noise import SH_OFFSETS, TAG_MAIN, spectral_noise, subharmonic_noise

# Table S1 (App. B): index-PSD power laws alpha = beta + 3 of characterised media.
MEDIA_ALPHA = {"atmosphere": 11.0 / 3.0, "ocean_min": 11.0 / 3.0, "ocean_max": 15.0 / 3.0,
               "tissue_min": 4.28, "tissue_max": 4.41}


def fried_parameter(wavelength, n0, cn2dz):
    """Eq. S18: r0 = [0.423 k^2 int Cn^2 dz]^(-3/5), k = 2 pi n0 / lambda."""
    k = 2.0 * np.pi * n0 / wavelength
    return (0.423 * k * k * np.asarray(cn2dz, dtype=np.float64)) ** (-3.0 / 5.0)


def psd_scales(l0, L0, inner_scale_conv=0):
    """(fm, f0) in cycles/m.  fm = inf when l0 <= 0, f0 = 0 when L0 is infinite or <= 0."""
    if l0 is None or l0 <= 0:
        fm = np.inf
    elif inner_scale_conv == 1:
        fm = 5.92 / (2.0 * np.pi * l0)
    else:
        fm = 1.0 / l0
    f0 = 0.0 if (L0 is None or not np.isfinite(L0) or L0 <= 0) else 1.0 / L0
    return fm, f0


def mvk_psd(f2, r0, fm, f0, alpha=11.0 / 3.0):
    """Eq. S17 in cycles/m; f2 = f^2.  Undefined (infinite) at f2 = 0 when f0 = 0.

    `alpha` generalises the power law to other media (App. B, Eq. S12/S15 and
    Table S1: the phase PSD of a medium with index PSD ~ kappa^-alpha falls as
    f^-alpha); the strength keeps the k^2 dz Cn^2 scaling of Eq. S15 through
    r0^(-5/3) = 0.423 k^2 cn2dz.  alpha = 11/3 is Eq. S17 itself."""
    f2 = np.asarray(f2, dtype=np.float64)
    inner = np.exp(-f2 / fm ** 2) if np.isfinite(fm) else 1.0
    with np.errstate(divide="ignore"):
        return 0.023 * r0 ** (-5.0 / 3.0) * inner / (f2 + f0 * f0) ** (alpha / 2.0)


def signed_bins(n):
    k = np.arange(n)
    return np.where(k < n // 2, k, k - n).astype(np.float64)


def psd_alpha(path):
    a = float(getattr(path, "psd_alpha", 0.0) or 0.0)
    return a if a > 0 else 11.0 / 3.0


def main_spectrum(n, dx, r0, fm, f0, noise, alpha=11.0 / 3.0):
    """Eq. S16 weighting: c = N_c * sqrt(W(f) df df); DC bin set to zero."""
    df = 1.0 / (n * dx)
    kh = signed_bins(n)
    f2 = (kh[:, None] ** 2 + kh[None, :] ** 2) * df * df
    w = mvk_psd(np.where(f2 > 0, f2, 1.0), r0, fm, f0, alpha)
    amp = np.sqrt(w) * df
    amp[0, 0] = 0.0
    return noise * amp


def unnormalised_idft(c):
    """z[i] = sum_k c[k] exp(+2 pi i k.i / N) (the inverse DFT of Eq. S16 without 1/N^2)."""
    n0, n1 = c.shape
    return np.fft.ifft2(c) * (n0 * n1)


def subharmonic_coefficients(n, dx, r0, fm, f0, sh_noise, alpha=11.0 / 3.0):
    """Eq. 2 weights: [levels][8] complex coefficients N_pq sqrt(W(f_pq)) df_p
    at the offsets SH_OFFSETS (m along y, n along x) of level p, df_p = df/3^p."""
    levels = sh_noise.shape[0]
    df = 1.0 / (n * dx)
    out = np.zeros((levels, 8), dtype=np.complex128)
    for p in range(1, levels + 1):
        dfp = df / 3.0 ** p
        for q, (m, nn) in enumerate(SH_OFFSETS):
            f2 = (m * m + nn * nn) * dfp * dfp
            out[p - 1, q] = sh_noise[p - 1, q] * np.sqrt(mvk_psd(f2, r0, fm, f0, alpha)) * dfp
    return out


def subharmonic_field(n, dx, coefs, x=None, y=None):
    """Eq. 2 sum: sum_pq c_pq exp(2 pi i (n df_p x + m df_p y)) on the centred
    grid, or at the given coordinate vectors x (columns) and y (rows)."""
    df = 1.0 / (n * dx)
    if x is None:
        x = (np.arange(n) - n // 2) * dx
    if y is None:
        y = (np.arange(n) - n // 2) * dx
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.zeros((len(y), len(x)), dtype=np.complex128)
    for p in range(1, coefs.shape[0] + 1):
        dfp = df / 3.0 ** p
        for q, (m, nn) in enumerate(SH_OFFSETS):
            z += coefs[p - 1, q] * np.exp(2j * np.pi * (nn * dfp * x[None, :] + m * dfp * y[:, None]))
    return z


def subharmonic_screen(n, dx, r0, fm, f0, sh_noise, alpha=11.0 / 3.0):
    """Eq. 2: complex subharmonic screen from [levels][8] noise coefficients."""
    return subharmonic_field(n, dx, subharmonic_coefficients(n, dx, r0, fm, f0, sh_noise, alpha))


def remove_piston(phi):
    """Subtract the mean over the grid (App. B, after Eq. S16)."""
    return phi - phi.mean()


def complex_screen(path, seed, t, pair, screen):
    """Complex screen z + z_SH for one realization pair and one screen (Eq. S16 + Eq. 2-3)."""
    n = int(path.n)
    r0 = fried_parameter(path.wavelength, path.n0, path.cn2dz[screen])
    fm, f0 = psd_scales(path.l0, path.L0, getattr(path, "inner_scale_conv", 0))
    alpha = psd_alpha(path)
    c = main_spectrum(n, path.dx, r0, fm, f0, spectral_noise(n, seed, t, pair, screen, TAG_MAIN), alpha)
    z = unnormalised_idft(c)
    levels = int(getattr(path, "sh_levels", 0))
    if levels > 0:
        z = z + subharmonic_screen(n, path.dx, r0, fm, f0,
                                   subharmonic_noise(levels, seed, t, pair, screen), alpha)
    return z


def split_pair(z):
    """Realizations 2j and 2j+1 from one complex screen, each with its piston removed."""
    return remove_piston(z.real), remove_piston(z.imag)


def phase_screens(path, seed, t=0):
    """All real screens, float64 [R][M][N][N] (radians)."""
    n, m, r = int(path.n), len(path.cn2dz), int(path.realizations)
    out = np.empty((r, m, n, n), dtype=np.float64)
    for j in range((r + 1) // 2):
        for s in range(m):
            a, b = split_pair(complex_screen(path, seed, t, j, s))
            out[2 * j, s] = a
            if 2 * j + 1 < r:
                out[2 * j + 1, s] = b
    return out
