"""Pins for the oracle's ensemble statistics (Sec. 3.2-3.3, Eq. S25)."""
import numpy as np

from oracle import stats


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
