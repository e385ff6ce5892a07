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


def summary(u, dx):
    """Returns dict(si_plane, w_2nd, w_fit, count) for a batch of fields."""
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
    return {"si_plane": float(si[central_mask(n)].mean()), "w_2nd": float(w2),
            "w_fit": float(wfit), "count": int(u.shape[0])}
