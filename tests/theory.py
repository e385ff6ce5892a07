"""Closed forms and exact expectations used to pin the oracle (test helpers).

Constants come from tests/golden/closed_forms.json, each cited to the paper.
The discrete expectations (structure function, first-order scintillation) are
sums over the grid's Fourier bins written independently of the synthesis code.
"""

import json
import os

import numpy as np

_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.json")
with open(_GOLDEN) as fh:
    CONST = {k: v["value"] for k, v in json.load(fh).items() if not k.startswith("_")}


def wavenumber(wavelength, n0=1.0):
    return 2.0 * np.pi * n0 / wavelength


def rytov_plane(cn2, wavelength, length, n0=1.0):
    """sigma_R^2 = 1.23 Cn^2 k^(7/6) L^(11/6) (App. C, Eq. S19/S26 for uniform Cn^2)."""
    k = wavenumber(wavelength, n0)
    return CONST["rytov_plane_wave_coefficient"] * cn2 * k ** (7.0 / 6.0) * length ** (11.0 / 6.0)


def si_all_regimes(s2):
    """Plane-wave SI for all regimes (App. C, Eq. S27, read with the 7/6 and 5/6 powers)."""
    a, b, c, d = CONST["strong_si"]
    s = s2 ** 0.5
    return np.exp(a * s2 / (1 + b * s ** (12.0 / 5.0)) ** (7.0 / 6.0)
                  + c * s2 / (1 + d * s ** (12.0 / 5.0)) ** (5.0 / 6.0)) - 1.0


def kolmogorov_structure(r, r0):
    return CONST["kolmogorov_structure_coefficient"] * (r / r0) ** (5.0 / 3.0)


def gaussian_vacuum(n, dx, w0, wavelength, z, n0=1.0):
    """Paraxial Gaussian beam of waist W0 at distance z (App. C, Eq. S22-S23 in
    field form): U = exp(-r^2 / (W0^2 q)) / q, q = 1 + i z / zR, zR = pi W0^2 n0 / lambda."""
    x = (np.arange(n) - n // 2) * dx
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    zr = np.pi * w0 * w0 * n0 / wavelength
    q = 1.0 + 1j * z / zr
    return np.exp(-r2 / (w0 * w0 * q)) / q


def gaussian_radius(w0, wavelength, z, n0=1.0):
    zr = np.pi * w0 * w0 * n0 / wavelength
    return w0 * np.sqrt(1.0 + (z / zr) ** 2)


def long_term_radius(w0, wavelength, z, sigma_r2, n0=1.0):
    """Weak-turbulence long-term radius W sqrt(1 + 1.33 sigma_R^2 Lambda^(5/6)),
    Lambda = 2 z / (k W^2) (App. C, Eq. S24, Andrews' weak form)."""
    w = gaussian_radius(w0, wavelength, z, n0)
    lam = 2.0 * z / (wavenumber(wavelength, n0) * w * w)
    return w * np.sqrt(1.0 + CONST["broadening_coefficient"] * sigma_r2 * lam ** (5.0 / 6.0))


def bin_frequencies(n, dx):
    df = 1.0 / (n * dx)
    k = np.arange(n)
    kh = np.where(k < n // 2, k, k - n).astype(np.float64)
    return kh[None, :] * df, kh[:, None] * df, df


def sh_frequencies(n, dx, levels):
    """(fx, fy, df_p) of every subharmonic point (3x3 grid without centre, df/3^p)."""
    df = 1.0 / (n * dx)
    out = []
    for p in range(1, levels + 1):
        dfp = df / 3.0 ** p
        for m in (-1, 0, 1):
            for q in (-1, 0, 1):
                if (m, q) != (0, 0):
                    out.append((q * dfp, m * dfp, dfp))
    return out


def structure_function_expected(n, dx, psd, rx, levels=0):
    """Exact E[(phi(x + rx) - phi(x))^2] along x for the discrete screens:
    2 sum_k W(f_k) df^2 (1 - cos 2 pi fx_k rx) + the same over subharmonic points."""
    fx, fy, df = bin_frequencies(n, dx)
    f2 = fx ** 2 + fy ** 2
    s = np.where(f2 > 0, psd(np.where(f2 > 0, f2, 1.0)) * df * df, 0.0)
    out = []
    for r in np.atleast_1d(rx):
        d = 2.0 * np.sum(s * (1.0 - np.cos(2 * np.pi * fx * r)))
        for (sx, sy, dfp) in sh_frequencies(n, dx, levels):
            d += 2.0 * psd(sx * sx + sy * sy) * dfp * dfp * (1.0 - np.cos(2 * np.pi * sx * r))
        out.append(d)
    return np.array(out)


def rytov_sum(n, dx, wavelength, dz, psds, n0=1.0):
    """First-order (Rytov) plane-wave scintillation of the discrete screens:
    SI = 4 sum_i sum_k W_i(f_k) df^2 sin^2(pi (lambda/n0) (L - z_i) f_k^2)."""
    fx, fy, df = bin_frequencies(n, dx)
    f2 = fx ** 2 + fy ** 2
    z = np.cumsum(dz[:-1])
    length = float(np.sum(dz))
    si = 0.0
    for zi, psd in zip(z, psds):
        s = np.where(f2 > 0, psd(np.where(f2 > 0, f2, 1.0)) * df * df, 0.0)
        si += 4.0 * np.sum(s * np.sin(np.pi * (wavelength / n0) * (length - zi) * f2) ** 2)
    return si
