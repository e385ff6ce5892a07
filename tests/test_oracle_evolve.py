"""Pins for the oracle's temporal evolution (Sec. 2.3 Eq. 4-5): exact translation
special cases and the AR(1) correlation law rho(tau) = alpha^tau (the calibration
quantity of Sec. 2.3, Fig. 3C)."""
import numpy as np

from oracle import evolve, screens
from paper_2604_07248_amd import workloads


def _path(n=32, r=2, m=1):
    return workloads.uniform_path(n, 0.5, 1e-6, 100.0 * m, m, 1e-13, 0.01, 10.0, 0, realizations=r)


def test_alpha_one_integer_shift_is_exact_roll():
    p = _path()
    c0 = evolve.initial_spectra(p, seed=1)
    phi0 = evolve.screens_from_spectra(c0, 2)
    c1 = evolve.evolve(c0, p, 1, 1, alpha=1.0, sx=3.0, sy=-2.0)
    phi1 = evolve.screens_from_spectra(c1, 2)
    assert np.max(np.abs(phi1 - np.roll(phi0, (-2, 3), axis=(-2, -1)))) < 1e-12 * np.abs(phi0).max()


def test_two_half_pixel_steps_equal_one_pixel():
    p = _path()
    c0 = evolve.initial_spectra(p, seed=2)
    half = evolve.evolve(evolve.evolve(c0, p, 2, 1, 1.0, 0.5, 0.5), p, 2, 2, 1.0, 0.5, 0.5)
    one = evolve.evolve(c0, p, 2, 1, 1.0, 1.0, 1.0)
    assert np.max(np.abs(half - one)) < 1e-12 * np.abs(one).max()


def test_static_initial_state_matches_static_screens():
    p = _path(r=4, m=2)
    c0 = evolve.initial_spectra(p, seed=5)
    assert np.allclose(evolve.screens_from_spectra(c0, 4), screens.phase_screens(p, 5), atol=1e-12)


def test_ar1_correlation_and_stationarity():
    """Zero shift: Pearson correlation of a screen with itself tau steps later is
    alpha^tau, and the variance per bin stays at W df^2 (Eq. 5's sqrt(1 - alpha^2))."""
    p = _path(n=32, r=48)
    alpha = 0.8
    c = evolve.initial_spectra(p, seed=3)
    phi0 = evolve.screens_from_spectra(c, p.realizations)
    var0 = np.mean(np.abs(c) ** 2)
    rho = []
    var = []
    for t in range(1, 7):
        c = evolve.evolve(c, p, 3, t, alpha, 0.0, 0.0)
        phi = evolve.screens_from_spectra(c, p.realizations)
        per = [np.corrcoef(a.ravel(), b.ravel())[0, 1] for a, b in zip(phi0[:, 0], phi[:, 0])]
        rho.append((np.mean(per), np.std(per, ddof=1) / np.sqrt(len(per))))
        var.append(np.mean(np.abs(c) ** 2) / var0)
    for tau, (r, se) in enumerate(rho, start=1):
        assert abs(r - alpha ** tau) < 4 * se + 0.01, (tau, r, alpha ** tau, se)
    assert np.all(np.abs(np.array(var) - 1) < 0.15), var


def test_nyquist_convention_and_dc():
    n = 8
    ph = evolve.shift_phase(n, 0.5, 0.0)
    assert np.isclose(ph[0, n // 2], np.exp(1j * np.pi / 2))   # k^ = -N/2
    p = _path(n=16)
    c1 = evolve.evolve(evolve.initial_spectra(p, 4), p, 4, 1, 0.5, 0.3, 0.7)
    assert np.all(c1[:, :, 0, 0] == 0)


def _sh_path(n=32, r=4, m=2, levels=3):
    return _path(n, r, m).with_(sh_levels=levels)


def test_sh_initial_state_matches_static_screens():
    """Main spectra and subharmonic coefficients at t = 0 give the static
    screens of Eq. S16 + Eq. 2-3 (same noise, same piston)."""
    p = _sh_path()
    c0, d0 = evolve.initial_spectra(p, seed=6), evolve.initial_sh(p, seed=6)
    assert np.allclose(evolve.screens_from_state(c0, d0, p, 4), screens.phase_screens(p, 6), atol=1e-12)


def test_sh_alpha_one_translates_the_subharmonic_field():
    """alpha = 1: the evolved coefficients describe the same Eq. 2 field
    translated by (sx, sy) pixels, for any real shift (the field is defined
    everywhere, not only on the periodic grid)."""
    p = _sh_path(n=32, r=2, m=1)
    d0 = evolve.initial_sh(p, seed=7)
    sx, sy = 0.7, -1.3
    d1 = evolve.evolve_sh(d0, p, 7, 1, alpha=1.0, sx=sx, sy=sy)
    x = (np.arange(p.n) - p.n // 2) * p.dx
    moved = screens.subharmonic_field(p.n, p.dx, d0[0, 0], x=x - sx * p.dx, y=x - sy * p.dx)
    got = screens.subharmonic_field(p.n, p.dx, d1[0, 0])
    assert np.max(np.abs(got - moved)) < 1e-12 * np.abs(moved).max()


def test_sh_alpha_zero_is_a_fresh_draw():
    p = _sh_path(n=32, r=2, m=1)
    d0 = evolve.initial_sh(p, seed=8)
    d1 = evolve.evolve_sh(d0, p, 8, 3, alpha=0.0, sx=0.3, sy=0.0)
    # same weights, different noise: the ratio to the static coefficient is not 1
    assert np.all(np.abs(d1) > 0) and not np.allclose(d1, d0)
    d1b = evolve.evolve_sh(d0 * 5.0, p, 8, 3, alpha=0.0, sx=0.0, sy=0.0)
    assert np.array_equal(d1, d1b)  # nothing of the old state survives


def test_sh_ar1_correlation_and_stationarity():
    """Zero shift: E[d_1 conj(d_0)] = alpha E|d_0|^2 and E|d_1|^2 = E|d_0|^2 =
    2 W(f_pq) df_p^2 (unit-variance real and imaginary parts), pooled over
    pairs and the 24 points after normalising by the weight."""
    alpha = 0.8
    p = _sh_path(n=32, r=512, m=1)
    d0 = evolve.initial_sh(p, seed=9)
    d1 = evolve.evolve_sh(d0, p, 9, 1, alpha=alpha, sx=0.0, sy=0.0)
    # the weight sqrt(W) df_p of each point: coefficient / noise of pair 0
    from oracle import noise
    wgt = np.abs(evolve._sh_coefficients(p, 9, 0, 0, 0, evolve.TAG_SH) / noise.subharmonic_noise(3, 9, 0, 0, 0))
    a0, a1 = d0[:, 0] / wgt, d1[:, 0] / wgt
    n = a0.size
    e0, e1 = np.mean(np.abs(a0) ** 2), np.mean(np.abs(a1) ** 2)
    assert abs(e0 - 2) < 4 * 2 / np.sqrt(n) and abs(e1 - 2) < 4 * 2 / np.sqrt(n)
    rho = np.mean((a1 * np.conj(a0)).real) / e0
    assert abs(rho - alpha) < 4 * np.sqrt((1 - alpha ** 2 + 1) / n)
