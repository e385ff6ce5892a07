"""Ensemble statistics of received fields, FP64 (Sec. 3.2-3.3, Eq. S25).

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

Over a batch of realizations of U [R][N][N], with I = |U|^2:
  m1 = <I>, m2 = <I^2> (population moments, 1/R);
  SI map  = m2 / m1^2 - 1 = sigma_I^2 / <I>^2 (Eq. S25);
  SI plane = mean of the SI map over the central region |x|, |y| < N dx / 4
             (pixels with |i - N/2| < N/4);
  W_2nd  = sqrt(2 sum r^2 m1 / sum m1)  (1/e^2 radius of a Gaussian from its
           second moment), r measured from pixel (N/2, N/2);
  W_fit  = least-squares fit of ln m1 = a - 2 r^2 / W^2 over pixels with
           m1 >= exp(-2) max m1 (the 1/e^2 intensity cutoff of Sec. 3.2).
Sec. 4.1 reads the scintillation of a beam over its power-cutoff region: the
per-pixel SI summed over the brightest pixels of the mean intensity that
together hold a fraction p (99.9 %) of its power.  That region is the pixels
with m1 >= the m1 of the k-th brightest pixel, k the fewest pixels whose
intensities reach p of the total (ties of the k-th value included).  Optional
weights (an aperture) multiply each pixel's SI and its count.
Moments are taken by the two-pass definition in FP64.
"""

import numpy as np


def moments(u):
    i = np.abs(np.asarray(u, dtype=np.complex128)) ** 2
    return i.mean(axis=0), (i * i).mean(axis=0)


def si_map(m1, m2):
    with np.errstate(divide="ignore", invalid="ignore"):
        return m2 / (m1 * m1) - 1.0


def central_mask(n):
    d = np.abs(np.arange(n) - n // 2)
    c = d < n // 4
    return c[:, None] & c[None, :]


def radius2(n, dx):
    x = (np.arange(n) - n // 2) * dx
    return x[None, :] ** 2 + x[:, None] ** 2


def power_cutoff_threshold(m1, fraction):
    """Intensity of the dimmest pixel in the power-cutoff region (Sec. 4.1):
    the brightest pixels, in decreasing m1, until their sum reaches
    `fraction` of the total."""
    v = np.sort(np.asarray(m1, dtype=np.float64).ravel())[::-1]
    k = int(np.searchsorted(np.cumsum(v), fraction * v.sum()))
    return float(v[min(k, v.size - 1)])


def region_si(si, m1, weight=None, power_fraction=0.0):
    """(weighted mean, weighted sum, weight total, threshold) of the SI map over
    the power-cutoff region (power_fraction > 0; threshold its dimmest
    intensity) or the central region (threshold 0)."""
    n = si.shape[-1]
    if power_fraction > 0:
        thr = power_cutoff_threshold(m1, power_fraction)
        sel = m1 >= thr
    else:
        thr = 0.0
        sel = central_mask(n)
    w = np.ones_like(si) if weight is None else np.asarray(weight, dtype=np.float64)
    tot = float(np.sum(w[sel]))
    ssum = float(np.sum((w * si)[sel]))
    return (ssum / tot if tot != 0 else 0.0), ssum, tot, thr


def summary(u, dx, weight=None, power_fraction=0.0):
    """Returns dict(si_plane, w_2nd, w_fit, count, si_sum, region_weight,
    threshold) for a batch of fields; the SI entries are taken over the
    region of region_si."""
    u = np.asarray(u)
    n = u.shape[-1]
    m1, m2 = moments(u)
    si = si_map(m1, m2)
    r2 = radius2(n, dx)
    w2 = np.sqrt(2.0 * np.sum(r2 * m1) / np.sum(m1))
    sel = m1 >= np.exp(-2.0) * m1.max()
    # ln m1 = a + b r^2, b = -2/W^2
    x, y = r2[sel], np.log(m1[sel])
    a_mat = np.stack([np.ones_like(x), x], axis=1)
    coef, *_ = np.linalg.lstsq(a_mat, y, rcond=None)
    wfit = np.sqrt(-2.0 / coef[1]) if coef[1] < 0 else np.inf
    mean, ssum, tot, thr = region_si(si, m1, weight, power_fraction)
    return {"si_plane": mean, "w_2nd": float(w2), "w_fit": float(wfit), "count": int(u.shape[0]),
            "si_sum": ssum, "region_weight": tot, "threshold": thr}
