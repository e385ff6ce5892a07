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
unnormalised inverse DFT, Re/Im pairing and piston removal.

With subharmonic levels the state also holds the Eq. 2 coefficients
d[p][q] of each pair and screen, evolved by the same two steps at their own
frequencies (n df_p, m df_p), df_p = df / 3^p:
  Eq. 4:  d <- d * exp(-2 pi i (n sx + m sy) / (3^p N)), the same translation
          by (sx, sy) pixels as the main spectrum;
  Eq. 5:  d <- alpha d + sqrt(1 - alpha^2) d_fresh, d_fresh drawn with the
          subharmonic AR tag at time t.
d_0 are the static coefficients (subharmonic tag, t = 0), so the initial
state reproduces the static screens of t = 0.
"""

import numpy as np

from .noise import SH_OFFSETS, TAG_AR, TAG_AR_SH, TAG_MAIN, TAG_SH, spectral_noise, subharmonic_noise
from .screens import (fried_parameter, main_spectrum, psd_alpha, psd_scales, remove_piston, signed_bins,
                      subharmonic_coefficients, subharmonic_field, unnormalised_idft, split_pair)


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


def _sh_coefficients(path, seed, t, pair, screen, tag):
    n = int(path.n)
    r0, fm, f0 = _psd_args(path, screen)
    noise = subharmonic_noise(int(path.sh_levels), seed, t, pair, screen, tag)
    return subharmonic_coefficients(n, path.dx, r0, fm, f0, noise, psd_alpha(path))


def initial_sh(path, seed):
    """[ceil(R/2)][M][levels][8] subharmonic coefficients at t = 0 (static, Eq. 2)."""
    p, m = (int(path.realizations) + 1) // 2, len(path.cn2dz)
    out = np.zeros((p, m, int(path.sh_levels), 8), dtype=np.complex128)
    for j in range(p):
        for s in range(m):
            out[j, s] = _sh_coefficients(path, seed, 0, j, s, TAG_SH)
    return out


def sh_shift_phase(n, levels, sx, sy):
    """[levels][8] Eq. 4 multipliers exp(-2 pi i (n sx + m sy) / (3^p N))."""
    out = np.zeros((levels, 8), dtype=np.complex128)
    for p in range(1, levels + 1):
        for q, (m, nn) in enumerate(SH_OFFSETS):
            out[p - 1, q] = np.exp(-2j * np.pi * (nn * sx + m * sy) / (3.0 ** p * n))
    return out


def evolve_sh(sh, path, seed, t, alpha, sx, sy):
    """One Eq. 4 + Eq. 5 step of every pair's and screen's subharmonic coefficients."""
    ph = sh_shift_phase(int(path.n), int(path.sh_levels), sx, sy)
    out = np.empty_like(sh)
    for j in range(sh.shape[0]):
        for s in range(sh.shape[1]):
            fresh = _sh_coefficients(path, seed, t, j, s, TAG_AR_SH)
            out[j, s] = alpha * (sh[j, s] * ph) + np.sqrt(1.0 - alpha * alpha) * fresh
    return out


def screens_from_state(spectra, sh, path, realizations):
    """Real screens [R][M][N][N] from pair spectra plus their subharmonic
    coefficients (Eq. 3), piston removed per realization."""
    p, m, n, _ = spectra.shape
    out = np.empty((realizations, m, n, n), dtype=np.float64)
    for j in range(p):
        for s in range(m):
            z = unnormalised_idft(spectra[j, s])
            if sh is not None and sh.shape[2] > 0:
                z = z + subharmonic_field(n, path.dx, sh[j, s])
            a, b = remove_piston(z.real), remove_piston(z.imag)
            out[2 * j, s] = a
            if 2 * j + 1 < realizations:
                out[2 * j + 1, s] = b
    return out
