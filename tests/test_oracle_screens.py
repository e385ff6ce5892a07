"""Pins for the oracle's phase-screen synthesis (App. B Eq. S16, App. C Eq. S17-S18,
Sec. 2.2 Eq. 2-3): brute-force DFT, exact PSD-recovery expectation (Sec. 3.1),
exact discrete structure function, and the Kolmogorov 6.88 (r/r0)^(5/3) law."""
import numpy as np
import pytest

from oracle import noise, screens
from paper_2604_07248_amd import workloads

import theory


def test_unnormalised_idft_matches_brute_force():
    rng = np.random.default_rng(0)
    n = 8
    c = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    i = np.arange(n)
    z = np.zeros((n, n), dtype=np.complex128)
    for k0 in range(n):
        for k1 in range(n):
            z += c[k0, k1] * np.exp(2j * np.pi * (k0 * i[:, None] + k1 * i[None, :]) / n)
    assert np.max(np.abs(screens.unnormalised_idft(c) - z)) < 1e-12 * np.max(np.abs(z))


def test_dc_zero_and_piston_removed():
    p = workloads.config1().path.with_(realizations=4)
    phi = screens.phase_screens(p, seed=3)
    assert np.max(np.abs(phi.mean(axis=(-1, -2)))) < 1e-12
    z = screens.complex_screen(p, 3, 0, 0, 0)
    # main part alone has an exactly zero mean (DC bin is zero)
    assert abs(z.mean()) < 1e-12 * np.abs(z).max()


def test_fried_parameter_scaling():
    # r0 ~ (k^2 Cn^2 dz)^(-3/5): doubling the integrated strength scales r0 by 2^(-3/5),
    # doubling the wavelength by 2^(6/5).
    r = screens.fried_parameter(1e-6, 1.0, np.array([1e-12, 2e-12]))
    assert np.isclose(r[1] / r[0], 2 ** -0.6, rtol=1e-13)
    r2 = screens.fried_parameter(2e-6, 1.0, 1e-12)
    assert np.isclose(r2 / r[0], 2 ** 1.2, rtol=1e-13)


def _pair_spectra(p, seed, count):
    out = []
    for j in range(count):
        a, b = screens.split_pair(screens.complex_screen(p, seed, 0, j, 0))
        out += [np.fft.fft2(a) / p.n ** 2, np.fft.fft2(b) / p.n ** 2]
    return np.array(out)


def test_psd_recovery_exact_expectation():
    """E |DFT(phi)[k] / N^2|^2 = W(f_k) df^2 for k != 0, for both members of a pair (Sec. 3.1)."""
    p = workloads.uniform_path(64, 0.5, 1e-6, 100.0, 1, 1e-13, 0.02, 5.0, 0, realizations=2)
    spec = _pair_spectra(p, seed=11, count=150)
    power = np.mean(np.abs(spec) ** 2, axis=0)
    r0 = screens.fried_parameter(p.wavelength, p.n0, p.cn2dz[0])
    fm, f0 = screens.psd_scales(p.l0, p.L0)
    fx, fy, df = theory.bin_frequencies(p.n, p.dx)
    f2 = fx ** 2 + fy ** 2
    expect = screens.mvk_psd(np.where(f2 > 0, f2, 1.0), r0, fm, f0) * df * df
    ratio = power / expect
    kr = np.sqrt(f2) / df
    checked = 0
    for lo, hi in [(0.5, 2), (2, 4), (4, 8), (8, 16), (16, 32)]:
        sel = (kr >= lo) & (kr < hi)
        # bins k and -k of a real screen are conjugate: half of them are independent
        n_ind = spec.shape[0] * max(sel.sum() // 2, 1)
        assert abs(ratio[sel].mean() - 1.0) < 4.0 / np.sqrt(n_ind), (lo, hi, ratio[sel].mean())
        checked += 1
    assert power[0, 0] < 1e-20
    # Re and Im members are uncorrelated
    cross = np.mean(spec[0::2] * np.conj(spec[1::2]), axis=0)
    assert np.abs(cross[kr > 0] / expect[kr > 0]).mean() < 0.2


def _structure(phis, lags):
    out = []
    # non-wrapping pairs only: subharmonic screens are not periodic on the grid
    for lag in lags:
        d = (phis[..., lag:] - phis[..., :-lag]) ** 2
        out.append(d.mean(axis=(-1, -2)))
    return np.array(out)  # [lags][screens]


@pytest.mark.parametrize("levels,alpha", [(0, 0.0), (3, 0.0), (3, 3.3), (2, 4.35)])
def test_structure_function_exact_discrete_expectation(levels, alpha):
    """Ensemble D(r) of the screens equals the exact discrete expectation
    2 sum W df^2 (1 - cos 2 pi f r) (+ subharmonic points, Eq. 2), for the
    Eq. S17 law and for other media power laws (App. B, Table S1)."""
    n, side = 128, 1.0
    p = workloads.Path(n=n, dx=side / n, wavelength=1e-6, dz=(0.0, 0.0), cn2dz=(1e-13,),
                       l0=0.0, L0=float("inf"), sh_levels=levels, realizations=2, psd_alpha=alpha)
    phis = []
    for j in range(60):
        a, b = screens.split_pair(screens.complex_screen(p, 21, 0, j, 0))
        phis += [a, b]
    phis = np.array(phis)
    lags = [1, 2, 4, 8, 16]
    est = _structure(phis, lags)
    r0 = screens.fried_parameter(p.wavelength, p.n0, p.cn2dz[0])
    fm, f0 = screens.psd_scales(p.l0, p.L0)
    a = screens.psd_alpha(p)
    expect = theory.structure_function_expected(n, p.dx, lambda f2: screens.mvk_psd(f2, r0, fm, f0, a),
                                                np.array(lags) * p.dx, levels)
    # pairs are independent; members of a pair are uncorrelated: use pair means for the SE
    pair_mean = 0.5 * (est[:, 0::2] + est[:, 1::2])
    se = pair_mean.std(axis=1, ddof=1) / np.sqrt(pair_mean.shape[1])
    assert np.all(np.abs(est.mean(axis=1) - expect) < 4.0 * se + 1e-12), (est.mean(axis=1), expect, se)


def test_structure_function_kolmogorov_band():
    """With l0 -> 0, L0 -> inf and three subharmonic levels, the discrete screens
    follow 6.88 (r/r0)^(5/3) at small separations (App. C PSD in cycles/m); without
    subharmonics the low-frequency deficit is much larger (Sec. 2.2)."""
    n, side = 256, 2.0
    cn2dz = 1e-12
    r0 = screens.fried_parameter(1e-6, 1.0, cn2dz)
    fm, f0 = screens.psd_scales(0.0, float("inf"))
    psd = lambda f2: screens.mvk_psd(f2, r0, fm, f0)  # noqa: E731
    dx = side / n
    lags = np.array([2, 4, 8, 16])
    with_sh = theory.structure_function_expected(n, dx, psd, lags * dx, levels=3)
    without = theory.structure_function_expected(n, dx, psd, lags * dx, levels=0)
    kolm = theory.kolmogorov_structure(lags * dx, r0)
    ratio_sh, ratio_no = with_sh / kolm, without / kolm
    assert np.all((ratio_sh > 0.80) & (ratio_sh < 1.05)), ratio_sh
    assert np.all(ratio_no < ratio_sh)
    assert ratio_no[-1] < 0.75
    # and the oracle's own screens reproduce the band (sampled)
    p = workloads.Path(n=n, dx=dx, wavelength=1e-6, dz=(0.0, 0.0), cn2dz=(cn2dz,), l0=0.0,
                       L0=float("inf"), sh_levels=3, realizations=2)
    phis = np.array([v for j in range(20) for v in screens.split_pair(screens.complex_screen(p, 5, 0, j, 0))])
    est = _structure(phis, lags).mean(axis=1) / kolm
    assert np.all((est > 0.7) & (est < 1.15)), est


def test_subharmonics_add_low_frequency_power_only():
    p = workloads.Path(n=64, dx=1.0 / 64, wavelength=1e-6, dz=(0.0, 0.0), cn2dz=(1e-13,), l0=0.01,
                       L0=50.0, sh_levels=3, realizations=2)
    z_sh = screens.complex_screen(p, 2, 0, 0, 0) - screens.complex_screen(p.with_(sh_levels=0), 2, 0, 0, 0)
    # a sum of frequencies at most df/3 per axis: the pixel-to-pixel change is bounded by
    # 2 pi (df/3) dx times the amplitude (sum of |coefficients|)
    amp = np.abs(z_sh - z_sh.mean()).max()
    step = max(np.abs(np.diff(z_sh, axis=0)).max(), np.abs(np.diff(z_sh, axis=1)).max())
    assert 0 < step <= 2 * np.pi / (3 * 64) * 2 * amp
    # level noise is drawn with the subharmonic tag, independent of the main spectrum
    assert not np.allclose(noise.subharmonic_noise(3, 2, 0, 0, 0)[0, :2],
                           noise.spectral_noise(64, 2, 0, 0, 0).ravel()[:2])


@pytest.mark.parametrize("alpha,slope,tol", [(3.3, 1.3, 0.05), (11.0 / 3.0, 5.0 / 3.0, 0.06),
                                             (4.35, 2.0, 0.06), (5.0, 2.0, 0.03)])
def test_media_power_law_structure_scaling(alpha, slope, tol):
    """A phase PSD ~ f^-alpha gives D(r) ~ r^(alpha-2) for 2 < alpha < 4 (App. B,
    Eq. S9-S11 projected to the screen) and a smooth screen, D ~ r^2, for
    alpha >= 4; checked on the exact discrete expectation with three
    subharmonic levels, l0 = 0, L0 = inf."""
    n, dx = 256, 2.0 / 256
    r0 = screens.fried_parameter(1e-6, 1.0, 1e-12)
    fm, f0 = screens.psd_scales(0.0, float("inf"))
    lags = np.array([2, 4, 8, 16])
    d = theory.structure_function_expected(n, dx, lambda f2: screens.mvk_psd(f2, r0, fm, f0, alpha), lags * dx, 3)
    fit = np.polyfit(np.log(lags), np.log(d), 1)[0]
    assert abs(fit - slope) < tol, (alpha, fit)


def test_default_power_law_is_eq_s17():
    f2 = np.array([0.5, 3.0, 40.0])
    assert np.array_equal(screens.mvk_psd(f2, 0.1, 100.0, 0.05), screens.mvk_psd(f2, 0.1, 100.0, 0.05, 11.0 / 3.0))
    p = workloads.config1().path
    assert screens.psd_alpha(p) == 11.0 / 3.0 and screens.psd_alpha(p.with_(psd_alpha=4.35)) == 4.35
