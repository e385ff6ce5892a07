"""Complex Gaussian noise N_c(0,1) for the phase-screen spectra (App. B Eq. S16,
Sec. 2.2 Eq. 2, Sec. 2.3 Eq. 5), drawn from Philox4x32-10 with a fixed counter
layout so that a given (seed, time step, realization pair, screen) always maps
to the same numbers.

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

Counter layout (the paper fixes no generator; this build's contract):
  key      = (seed mod 2^32, seed >> 32)
  counter  = (e, t, j, (tag << 28) | s)
    t   time step (0 for static screens and for the initial AR spectrum)
    j   realization-pair index (realizations 2j and 2j+1 share one complex screen)
    s   screen index along the path
    tag 1 = main spectrum, 2 = subharmonics, 3 = AR innovation, 4 = AR innovation
    of the subharmonic coefficients
  main / AR spectrum of an N x N grid: e = k0*N + k1 for 0 <= k0 < N/2; words
    (v0, v1) give bin (k0, k1) and words (v2, v3) give bin (k0 + N/2, k1).
  subharmonics: level p (1-based), offset index q in 0..7 over the 3x3 grid
    without its centre (row-major, row = y offset m, column = x offset n):
    e = 4*(p-1) + q//2; even q uses (v0, v1), odd q uses (v2, v3).
Uniform map u(v) = (floor(v / 512) + 1/2) * 2^-23, in (0, 1), exact in FP32
(24 significant bits), so both sides of a comparison start from the same u.
Box-Muller: rho = sqrt(-2 ln u(va)), theta = 2 pi u(vb),
N_c = rho cos(theta) + i rho sin(theta); real and imaginary parts are each
N(0, 1) (unit variance per component, the reading under which Parseval holds for
Eq. S16).
"""

import numpy as np

from .philox import philox4x32_10

TAG_MAIN = 1
TAG_SH = 2
TAG_AR = 3
TAG_AR_SH = 4

# 3x3 sub-grid offsets (m = y offset, n = x offset) without the centre, Eq. 2.
SH_OFFSETS = [(m, n) for m in (-1, 0, 1) for n in (-1, 0, 1) if (m, n) != (0, 0)]


def seed_key(seed):
    seed = int(seed)
    return (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def counters(e, t, pair, tag, screen):
    e = np.asarray(e, dtype=np.uint64)
    out = np.empty(e.shape + (4,), dtype=np.uint64)
    out[..., 0] = e
    out[..., 1] = int(t) & 0xFFFFFFFF
    out[..., 2] = int(pair) & 0xFFFFFFFF
    out[..., 3] = ((int(tag) << 28) | int(screen)) & 0xFFFFFFFF
    return out


def uniform_open01(v):
    """u(v) = (floor(v/512) + 0.5) / 2^23."""
    v = np.asarray(v, dtype=np.uint64)
    return ((v >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(va, vb):
    rho = np.sqrt(-2.0 * np.log(uniform_open01(va)))
    theta = 2.0 * np.pi * uniform_open01(vb)
    return rho * np.cos(theta) + 1j * rho * np.sin(theta)


def spectral_noise(n, seed, t, pair, screen, tag=TAG_MAIN):
    """N x N complex noise for the main (or AR innovation) spectrum."""
    assert n % 2 == 0
    h = n // 2
    e = np.arange(h, dtype=np.uint64)[:, None] * np.uint64(n) + np.arange(n, dtype=np.uint64)[None, :]
    v = philox4x32_10(counters(e, t, pair, tag, screen), seed_key(seed))
    out = np.empty((n, n), dtype=np.complex128)
    out[:h] = box_muller(v[..., 0], v[..., 1])
    out[h:] = box_muller(v[..., 2], v[..., 3])
    return out


def subharmonic_noise(levels, seed, t, pair, screen, tag=TAG_SH):
    """[levels][8] complex noise for the subharmonic coefficients of Eq. 2
    (tag TAG_AR_SH: the innovations of their AR evolution)."""
    out = np.zeros((levels, 8), dtype=np.complex128)
    for p in range(1, levels + 1):
        e = np.array([4 * (p - 1) + q for q in range(4)], dtype=np.uint64)
        v = philox4x32_10(counters(e, t, pair, tag, screen), seed_key(seed))
        for q in range(8):
            w = v[q // 2]
            out[p - 1, q] = box_muller(w[0], w[1]) if q % 2 == 0 else box_muller(w[2], w[3])
    return out
