"""Screen placement along a path, FP64 (Sec. 2.4, Eq. 7; App. C Eq. S18-S21).

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

Readings (listed in the design notes):
  * The strength of an interval [a, b] is Eq. S19 applied to it:
        s2(a, b) = 3.27 k^(7/6) D^(5/6) int_a^b Cn2(z) (1 - (z - a)/D)^(5/3) dz,
    D = b - a, k = 2 pi n0 / lambda.
  * Sec. 2.4's routine, in its order: (1) start from the user's intervals
    (M0 equal ones by default); (2) halve every interval whose s2 exceeds the
    limit, until none does; (3) merge neighbours, left to right, whenever the
    merged interval stays within the limit; (4) "linear fit": keep the count M
    and move the interior boundaries to where the cumulative strength,
    interpolated linearly between the rough boundaries, reaches j/M of its
    total, then halve again any interval above the limit; (5) halve every
    interval longer than the Eq. 7 step.
  * Eq. 7 as derived in the text (the printed fraction is inverted):
    dz_max = (N dx / 2) sqrt(n0^2 k0^2 - kappa0^2) / kappa0, kappa0 = 2 pi / dx,
    k0 = 2 pi / lambda; about N dx^2 n0 / (2 lambda) for dx >> lambda.
  * One screen at the middle of each interval; the diffraction distances are
    [D_0/2, (D_0 + D_1)/2, ..., D_(M-1)/2] and the screen's integrated
    strength is int Cn2 dz over its interval.
  * Eq. S21 (Hufnagel-Valley) with z the height above the ground, the source
    at the ground and the path running vertically upward.
Integrals use scipy's adaptive quadrature.
"""

import numpy as np
from scipy import integrate


def hufnagel_valley(z, A=1.7e-14, V=21.0):
    """Eq. S21: Cn2(z) for height z [m], ground constant A, wind speed V."""
    z = np.asarray(z, dtype=np.float64)
    return (0.00594 * (V / 27.0) ** 2 * (1e-5 * z) ** 10 * np.exp(-z / 1000.0)
            + 2.7e-16 * np.exp(-z / 1500.0) + A * np.exp(-z / 100.0))


def table_profile(z, values):
    """Cn2 piecewise linear through (z[i], values[i]), constant beyond the ends."""
    z = np.asarray(z, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)

    def cn2(h):
        return np.interp(h, z, v)
    cn2.nodes = z
    return cn2


def _quad(f, a, b, cn2=None):
    nodes = getattr(cn2, "nodes", None)
    pts = None
    if nodes is not None:
        inside = [float(x) for x in nodes if a < x < b]
        pts = inside or None
    return integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-12, limit=400, points=pts)[0]


def wavenumber(wavelength, n0=1.0):
    return 2.0 * np.pi * n0 / wavelength


def rytov_interval(cn2, a, b, wavelength, n0=1.0):
    """Eq. S19 over [a, b]."""
    d = b - a
    k = wavenumber(wavelength, n0)
    w = _quad(lambda z: float(cn2(z)) * (1.0 - (z - a) / d) ** (5.0 / 3.0), a, b, cn2)
    return 3.27 * k ** (7.0 / 6.0) * d ** (5.0 / 6.0) * w


def integrated_cn2(cn2, a, b):
    return _quad(lambda z: float(cn2(z)), a, b, cn2)


def fried_interval(cn2, a, b, wavelength, n0=1.0):
    """Eq. S18 over [a, b]."""
    k = wavenumber(wavelength, n0)
    return (0.423 * k * k * integrated_cn2(cn2, a, b)) ** (-3.0 / 5.0)


def fried_weak_limit(cn2, a, b, wavelength, n0=1.0):
    """Eq. S20: the interval's r0 at which its Rytov variance (Eq. S19) is 1."""
    d = b - a
    k = wavenumber(wavelength, n0)
    w = _quad(lambda z: float(cn2(z)) * (1.0 - (z - a) / d) ** (5.0 / 3.0), a, b, cn2)
    ratio = w / integrated_cn2(cn2, a, b)
    return (0.129 * k ** (5.0 / 6.0) / d ** (5.0 / 6.0) / ratio) ** (-3.0 / 5.0)


def aliasing_step(n, dx, wavelength, n0=1.0):
    """Eq. 7 (with the fraction as derived in Sec. 2.4)."""
    k0 = 2.0 * np.pi / wavelength
    kap = 2.0 * np.pi / dx
    arg = n0 * n0 * k0 * k0 - kap * kap
    if arg <= 0:
        raise ValueError("dx below lambda / n0: Eq. 7 has no real step")
    return 0.5 * n * dx * np.sqrt(arg) / kap


def _split(bounds, too_big):
    out = [bounds[0]]
    for b in bounds[1:]:
        a = out[-1]
        stack = [(a, b)]
        while stack:
            lo, hi = stack.pop()
            if too_big(lo, hi):
                mid = 0.5 * (lo + hi)
                stack.append((mid, hi))
                stack.append((lo, mid))
            else:
                out.append(hi)
    return out


def place_screens(cn2, length, wavelength, n, dx, rytov_limit, initial=1, n0=1.0):
    """Sec. 2.4's placement.  `initial`: a count of equal intervals or a list of
    interior boundaries.  Returns a dict with the interval boundaries, the
    diffraction distances dz [M+1], the integrated strengths cn2dz [M], and per
    interval its Rytov variance and Fried parameter."""
    if rytov_limit <= 0:
        raise ValueError("rytov_limit must be positive")
    if np.isscalar(initial):
        bounds = list(np.linspace(0.0, length, int(initial) + 1))
    else:
        bounds = [0.0] + sorted(float(x) for x in initial) + [float(length)]
    s2 = lambda a, b: rytov_interval(cn2, a, b, wavelength, n0)
    over = lambda a, b: s2(a, b) > rytov_limit
    # (2) split
    bounds = _split(bounds, over)
    # (3) merge neighbours, left to right
    merged = [bounds[0], bounds[1]]
    for b in bounds[2:]:
        if s2(merged[-2], b) <= rytov_limit:
            merged[-1] = b
        else:
            merged.append(b)
    bounds = merged
    # (4) linear fit on the cumulative strength: boundary j goes where the
    # cumulative s2, linear within each interval, reaches j/M of the total (in
    # the first interval whose end reaches it); then split again
    m = len(bounds) - 1
    if m > 1:
        cum = [0.0]
        for i in range(m):
            cum.append(cum[-1] + s2(bounds[i], bounds[i + 1]))
        new = [0.0]
        for j in range(1, m):
            target = cum[m] * j / m
            i = 0
            while i + 1 < m and cum[i + 1] < target:
                i += 1
            span = cum[i + 1] - cum[i]
            frac = (target - cum[i]) / span if span > 0 else 0.0
            new.append(bounds[i] + frac * (bounds[i + 1] - bounds[i]))
        bounds = new + [float(length)]
        bounds = _split(bounds, over)
    # (5) Eq. 7
    dzmax = aliasing_step(n, dx, wavelength, n0)
    bounds = _split(bounds, lambda a, b: (b - a) > dzmax)
    bounds = np.asarray(bounds, dtype=np.float64)
    widths = np.diff(bounds)
    dz = np.concatenate([[0.5 * widths[0]], 0.5 * (widths[:-1] + widths[1:]), [0.5 * widths[-1]]])
    cn2dz = np.array([integrated_cn2(cn2, bounds[i], bounds[i + 1]) for i in range(len(widths))])
    return {"bounds": bounds, "dz": dz, "cn2dz": cn2dz,
            "rytov": np.array([s2(bounds[i], bounds[i + 1]) for i in range(len(widths))]),
            "r0": np.array([fried_interval(cn2, bounds[i], bounds[i + 1], wavelength, n0)
                            for i in range(len(widths))]),
            "dz_max": dzmax}
