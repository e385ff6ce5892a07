"""Pins for the oracle's ensemble statistics (Sec. 3.2-3.3, Eq. S25)."""
import numpy as np

import pytest

from oracle import stats
from oracle import stats as ost


def _welford(fields):
    """Streaming mean/second moment (Welford's update, Sec. 3.3)."""
    n = 0
    mean = np.zeros(fields.shape[1:])
    m2 = np.zeros(fields.shape[1:])
    for f in fields:
        i = np.abs(f) ** 2
        n += 1
        d = i - mean
        mean += d / n
        m2 += d * (i - mean)
    return mean, m2 / n


def test_two_pass_equals_welford():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((37, 16, 16)) + 1j * rng.standard_normal((37, 16, 16))
    m1, m2 = stats.moments(u)
    wm, wv = _welford(u)
    assert np.allclose(m1, wm, rtol=1e-12)
    assert np.allclose(m2 - m1 ** 2, wv, rtol=1e-10)
    si = stats.si_map(m1, m2)
    assert np.allclose(si, wv / wm ** 2, rtol=1e-10)


def test_constant_field_has_zero_scintillation():
    u = np.full((8, 16, 16), 2.0 + 1.0j)
    s = stats.summary(u, 0.01)
    assert abs(s["si_plane"]) < 1e-14


def test_fully_developed_speckle_has_unit_si():
    rng = np.random.default_rng(1)
    u = rng.standard_normal((400, 32, 32)) + 1j * rng.standard_normal((400, 32, 32))
    m1, m2 = stats.moments(u)
    si = stats.si_map(m1, m2)
    # exponential intensity: SI = 1; per-pixel SE ~ sqrt(20/400) -> plane mean over 1024 px
    assert abs(si.mean() - 1.0) < 4 * np.sqrt(20.0 / 400) / np.sqrt(1024) + 0.01


def test_radius_estimators_on_exact_gaussian():
    n, dx, w = 128, 0.002, 0.03
    x = (np.arange(n) - n // 2) * dx
    u = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / w ** 2)[None]
    s = stats.summary(u, dx)
    assert abs(s["w_fit"] / w - 1) < 1e-10
    assert abs(s["w_2nd"] / w - 1) < 1e-3


def test_power_cutoff_region_is_minimal_brute_force():
    """Sec. 4.1 region: the fewest brightest pixels whose intensities reach the
    fraction; checked against every prefix of the sorted values."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        m1 = rng.exponential(size=(6, 6))
        for p in (0.5, 0.9, 0.999, 1.0):
            thr = ost.power_cutoff_threshold(m1, p)
            inside = m1[m1 >= thr].sum()
            assert inside >= p * m1.sum() * (1 - 1e-15)
            dimmer_removed = m1[m1 > thr].sum()
            assert dimmer_removed < p * m1.sum()


def test_power_cutoff_of_gaussian_beam_closed_form():
    """A Gaussian exp(-2 r^2 / W^2) holds 1 - exp(-2 R^2 / W^2) of its power
    inside radius R, so the 99.9 % region ends where the intensity is 1e-3 of
    the peak, at R = W sqrt(ln(1000) / 2)."""
    n, dx, w = 256, 1.0, 24.0
    x = (np.arange(n) - n // 2) * dx
    m1 = np.exp(-2 * (x[None, :] ** 2 + x[:, None] ** 2) / w ** 2)
    thr = ost.power_cutoff_threshold(m1, 0.999)
    assert thr / m1.max() == pytest.approx(1e-3, rel=0.03)
    area = (m1 >= thr).sum() * dx * dx
    assert area == pytest.approx(np.pi * w * w * np.log(1000.0) / 2, rel=0.01)


def test_region_si_weights_and_central_default():
    n = 16
    si = np.arange(n * n, dtype=np.float64).reshape(n, n)
    m1 = np.ones((n, n))
    mean, ssum, tot, thr = ost.region_si(si, m1)
    c = ost.central_mask(n)
    assert thr == 0.0 and tot == c.sum() and ssum == si[c].sum() and mean == si[c].mean()
    w = np.zeros((n, n))
    w[n // 2, n // 2] = 2.0
    mean, ssum, tot, _ = ost.region_si(si, m1, weight=w, power_fraction=1.0)
    assert tot == 2.0 and mean == si[n // 2, n // 2] and ssum == 2 * si[n // 2, n // 2]
