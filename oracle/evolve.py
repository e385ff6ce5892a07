"""Temporal evolution of stored screen spectra, FP64 (Sec. 2.3 Eq. 4-5).

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

The state is the complex spectrum c_t[k0][k1] of one realization pair and one
screen (Eq. S16 weighting, DC zero).  One time step (Sec. 2.3: translate first,
then blend in fresh PSD-weighted noise):
  Eq. 4 (frozen flow):  c <- c * exp(-2 pi i (k1^ sx + k0^ sy) / N), a shift of
        the screen by (sx, sy) pixels, sx = T vx / dx.  The Nyquist bin uses
        k^ = -N/2.
  Eq. 5 (AR(1) boiling): c <- alpha c + sqrt(1 - alpha^2) sqrt(W df^2) N_c,
        N_c drawn with the AR innovation tag at time step t (t >= 1).
The initial state c_0 is the static main spectrum (tag main, t = 0), so the
stationary variance W df^2 holds at every t.  Screens come from c_t by the
unnormalised inverse DFT, Re/Im pairing and piston removal, without
subharmonics.
"""

import numpy as np

from .noise import TAG_AR, TAG_MAIN, spectral_noise
from .screens import fried_parameter, main_spectrum, psd_alpha, psd_scales, signed_bins, split_pair, unnormalised_idft


def _psd_args(path, screen):
    r0 = fried_parameter(path.wavelength, path.n0, path.cn2dz[screen])
    fm, f0 = psd_scales(path.l0, path.L0, getattr(path, "inner_scale_conv", 0))
    return r0, fm, f0


def initial_spectrum(path, seed, pair, screen):
    n = int(path.n)
    r0, fm, f0 = _psd_args(path, screen)
    return main_spectrum(n, path.dx, r0, fm, f0, spectral_noise(n, seed, 0, pair, screen, TAG_MAIN), psd_alpha(path))


def shift_phase(n, sx, sy):
    """Eq. 4 multiplier exp(-2 pi i (k1^ sx + k0^ sy)/N) on the natural-order grid."""
    kh = signed_bins(n)
    return np.exp(-2j * np.pi * (kh[None, :] * sx + kh[:, None] * sy) / n)


def evolve_step(c_prev, path, seed, t, pair, screen, alpha, sx, sy):
    """One AR(1) + frozen-flow step (t >= 1), Eq. 4 then Eq. 5."""
    n = int(path.n)
    r0, fm, f0 = _psd_args(path, screen)
    fresh = main_spectrum(n, path.dx, r0, fm, f0, spectral_noise(n, seed, t, pair, screen, TAG_AR), psd_alpha(path))
    return alpha * (c_prev * shift_phase(n, sx, sy)) + np.sqrt(1.0 - alpha * alpha) * fresh


def initial_spectra(path, seed):
    """[ceil(R/2)][M][N][N] complex initial state."""
    n, m, r = int(path.n), len(path.cn2dz), int(path.realizations)
    out = np.empty(((r + 1) // 2, m, n, n), dtype=np.complex128)
    for j in range(out.shape[0]):
        for s in range(m):
            out[j, s] = initial_spectrum(path, seed, j, s)
    return out


def evolve(spectra, path, seed, t, alpha, sx, sy):
    out = np.empty_like(spectra)
    for j in range(spectra.shape[0]):
        for s in range(spectra.shape[1]):
            out[j, s] = evolve_step(spectra[j, s], path, seed, t, j, s, alpha, sx, sy)
    return out


def screens_from_spectra(spectra, realizations):
    """Real screens [R][M][N][N] from pair spectra (no subharmonics in the AR state)."""
    p, m, n, _ = spectra.shape
    out = np.empty((realizations, m, n, n), dtype=np.float64)
    for j in range(p):
        for s in range(m):
            a, b = split_pair(unnormalised_idft(spectra[j, s]))
            out[2 * j, s] = a
            if 2 * j + 1 < realizations:
                out[2 * j + 1, s] = b
    return out
