"""Pins of the oracle's screen placement (Sec. 2.4, Eq. 7; App. C Eq. S18-S21)."""
import math

import numpy as np
import pytest

from oracle import planner as opl

LAM = 1.064e-6


def uniform(c):
    return lambda z: c


def test_uniform_interval_rytov_closed_form():
    """Eq. S19 with constant Cn2: the weight integrates to 3/8 of the length,
    so s2 = 3.27 * 3/8 * Cn2 k^(7/6) D^(11/6)."""
    c, a, b = 3e-15, 250.0, 1900.0
    k = 2 * math.pi / LAM
    want = 3.27 * 0.375 * c * k ** (7 / 6) * (b - a) ** (11 / 6)
    assert opl.rytov_interval(uniform(c), a, b, LAM) == pytest.approx(want, rel=1e-10)


def test_hufnagel_valley_integral_and_r0():
    """Eq. S21 integrates in closed form over [0, inf):
    0.00594 (V/27)^2 1e-50 10! 1000^11 + 2.7e-16 * 1500 + A * 100, and the
    standard HV 5/7 profile (A = 1.7e-14, V = 21) has r0 of about 5 cm at
    500 nm looking up from the ground (its name)."""
    A, V = 1.7e-14, 21.0
    closed = 0.00594 * (V / 27) ** 2 * 1e-50 * math.factorial(10) * 1000.0 ** 11 + 2.7e-16 * 1500 + A * 100
    cn2 = lambda z: opl.hufnagel_valley(z, A, V)
    total = sum(opl.integrated_cn2(cn2, a, b) for a, b in ((0, 1e3), (1e3, 2e4), (2e4, 1e5), (1e5, 3e5)))
    assert total == pytest.approx(closed, rel=1e-9)
    r0 = (0.423 * (2 * math.pi / 0.5e-6) ** 2 * total) ** (-3 / 5)
    assert 0.048 < r0 < 0.052
    assert float(opl.hufnagel_valley(0.0, A, V)) == pytest.approx(A + 2.7e-16, rel=1e-15)


@pytest.mark.parametrize("prof", ["uniform", "hv"])
def test_weak_limit_r0_identity(prof):
    """Eq. S20 follows from Eq. S18 and S19 at s2 = 1: for any interval
    r0_S20 = r0_S18 (0.423 / (0.129 * 3.27) s2)^(3/5) (0.129 is 0.423/3.27 rounded)."""
    cn2 = uniform(2e-14) if prof == "uniform" else (lambda z: opl.hufnagel_valley(z, 1e-13))
    a, b = 30.0, 1530.0
    s2 = opl.rytov_interval(cn2, a, b, LAM)
    r18 = opl.fried_interval(cn2, a, b, LAM)
    r20 = opl.fried_weak_limit(cn2, a, b, LAM)
    assert r20 == pytest.approx(r18 * (0.423 / (0.129 * 3.27) * s2) ** 0.6, rel=1e-10)


def test_aliasing_step_paraxial_limit():
    """Eq. 7 tends to N dx^2 n0 / (2 lambda) when dx >> lambda."""
    n, dx = 1024, 1e-3
    assert opl.aliasing_step(n, dx, LAM) == pytest.approx(n * dx * dx / (2 * LAM), rel=1e-6)
    with pytest.raises(ValueError):
        opl.aliasing_step(64, 0.5e-6, LAM)


@pytest.mark.parametrize("ratio", [0.5, 1.5, 7.0, 40.0])
def test_uniform_path_screen_count(ratio):
    """Constant Cn2: halving gives 2^p equal intervals with p the least integer
    for which one piece is within the limit; merging two pieces would exceed
    it, and the linear fit keeps equal pieces equal."""
    c, L = 1e-14, 2000.0
    s2_total = opl.rytov_interval(uniform(c), 0.0, L, LAM)
    limit = s2_total / ratio
    p = max(0, math.ceil(math.log2(ratio ** (6 / 11)) - 1e-12))
    res = opl.place_screens(uniform(c), L, LAM, n=4096, dx=2e-3, rytov_limit=limit)
    assert len(res["cn2dz"]) == 2 ** p
    np.testing.assert_allclose(np.diff(res["bounds"]), L / 2 ** p, rtol=1e-12)
    assert res["dz"][0] == pytest.approx(L / 2 ** (p + 1), rel=1e-12)


def test_aliasing_split_count():
    """Negligible turbulence on a path of 5 Eq.-7 steps: halving reaches
    L/8 < dz_max < L/4, so 8 screens, one every L/8."""
    n, dx = 256, 1e-3
    dzmax = opl.aliasing_step(n, dx, LAM)
    L = 5 * dzmax
    res = opl.place_screens(uniform(1e-20), L, LAM, n=n, dx=dx, rytov_limit=1.0)
    assert len(res["cn2dz"]) == 8
    np.testing.assert_allclose(res["dz"], [L / 16] + [L / 8] * 7 + [L / 16], rtol=1e-12)


@pytest.mark.parametrize("A,L,limit", [(1.7e-14, 3000.0, 0.05), (1e-13, 5000.0, 0.1), (1e-12, 1500.0, 0.2)])
def test_hufnagel_valley_placement_invariants(A, L, limit):
    cn2 = lambda z: opl.hufnagel_valley(z, A)
    n, dx = 1024, 1e-3
    res = opl.place_screens(cn2, L, LAM, n=n, dx=dx, rytov_limit=limit, initial=4)
    w = np.diff(res["bounds"])
    assert np.all(w > 0) and res["bounds"][0] == 0.0 and res["bounds"][-1] == pytest.approx(L, rel=1e-14)
    assert np.all(res["rytov"] <= limit * (1 + 1e-12))
    assert np.all(w <= res["dz_max"] * (1 + 1e-12))
    assert res["dz"].sum() == pytest.approx(L, rel=1e-12)
    assert res["cn2dz"].sum() == pytest.approx(opl.integrated_cn2(cn2, 0.0, L), rel=1e-9)
    # r0 per screen is Eq. S18 of its integrated strength
    k = 2 * math.pi / LAM
    np.testing.assert_allclose(res["r0"], (0.423 * k * k * res["cn2dz"]) ** -0.6, rtol=1e-12)


def test_linear_fit_evens_out_strength():
    """The linear fit moves boundaries toward equal strength: on a profile with
    a steep ground layer the spread of per-interval s2 after placement is below
    that of the split/merge pieces it starts from."""
    cn2 = lambda z: opl.hufnagel_valley(z, 5e-13)
    L, limit = 4000.0, 0.1
    res = opl.place_screens(cn2, L, LAM, n=8192, dx=2e-3, rytov_limit=limit, initial=1)
    s2 = res["rytov"]
    # rough pieces: halving alone
    rough = opl._split([0.0, L], lambda a, b: opl.rytov_interval(cn2, a, b, LAM) > limit)
    s2_rough = np.array([opl.rytov_interval(cn2, rough[i], rough[i + 1], LAM) for i in range(len(rough) - 1)])
    assert s2.max() / s2.min() < s2_rough.max() / s2_rough.min()


def test_rejects_bad_limit():
    with pytest.raises(ValueError):
        opl.place_screens(uniform(1e-14), 100.0, LAM, 256, 1e-3, 0.0)


def test_table_profile_ramp_closed_form():
    """Cn2 linear in z through two table points: int Cn2 = c0 D + c1 (b^2 - a^2)/2
    and, since int_0^1 t (1-t)^(5/3) dt = B(2, 8/3) = 9/88, Eq. S19's weighted
    integral is (c0 + c1 a) D 3/8 + c1 D^2 9/88."""
    c0, c1, a, b = 2e-15, 3e-18, 100.0, 2600.0
    prof = opl.table_profile([0.0, 5000.0], [c0, c0 + c1 * 5000.0])
    d = b - a
    assert opl.integrated_cn2(prof, a, b) == pytest.approx(c0 * d + c1 * (b * b - a * a) / 2, rel=1e-12)
    k = 2 * math.pi / LAM
    w = (c0 + c1 * a) * d * 0.375 + c1 * d * d * 9 / 88
    assert opl.rytov_interval(prof, a, b, LAM) == pytest.approx(3.27 * k ** (7 / 6) * d ** (5 / 6) * w, rel=1e-10)
    # beyond the table the profile is constant
    assert float(prof(6000.0)) == pytest.approx(c0 + c1 * 5000.0)
