"""Closed-form pins of the oracle's PSD (App. C Eq. S17-S18, App. B Eq. S12/S15)
and of its screens through the propagation (Sec. 2.1 Eq. 1).

Each factor of the modified von Karman PSD is checked against mathematics that
does not evaluate the oracle's formula:
  * outer scale: on a lattice fine against 1/L0 with no inner scale, the summed
    phase variance sum_k W(f_k) df^2 equals the integral
    0.023 r0^(-5/3) (6 pi / 5) L0^(5/3);
  * inner and outer scale together, any power law alpha: the variance and the
    phase-gradient variance sum_k 4 pi^2 f_k^2 W(f_k) df^2 equal their
    integrals, which reduce to Tricomi's confluent hypergeometric function
    U(a, b, z) (scipy.special.hyperu):
        variance  = 0.023 r0^(-5/3) pi c^(1 - alpha/2) U(1, 2 - alpha/2, c/fm^2)
        gradient  = 0.023 r0^(-5/3) 4 pi^3 c^(2 - alpha/2) U(2, 3 - alpha/2, c/fm^2)
    with c = f0^2 (substitute u = f^2 = c t in the radial integral).  The lattice
    sum of a function analytic near the real axis converges exponentially in
    f0/df (Poisson summation), so the agreement is at rounding level;
  * the inner-scale conventions: the Gaussian factor of W falls to 1/e at
    kappa = 2 pi / l0 rad/m (Eq. S17 as printed) or at kappa = 5.92 / l0
    (inner_scale_conv = 1);
  * the beam second-moment invariant: a screen at z_i adds E|grad phi_i|^2 / k^2
    to the mean square angle of the beam and nothing to <r^2> or <r . theta>
    (the screen is independent of the field reaching it), so at the receiver
      E<r^2> - <r^2>_vac = sum_i (L - z_i)^2 sum_k 4 pi^2 f_k^2 S_ik / k^2,
    S_ik = W_i(f_k) df^2, checked on an oracle ensemble within 4 standard errors.
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import propagate as opr
from oracle import screens as osc
from paper_2604_07248_amd import workloads


def _lattice_f2(n, df):
    k = np.arange(n)
    kh = np.where(k < n // 2, k, k - n).astype(np.float64)
    return (kh[:, None] ** 2 + kh[None, :] ** 2) * df * df


def test_outer_scale_phase_variance_closed_form():
    """l0 = 0 (no inner scale): sum_k W df^2 = 0.023 r0^(-5/3) (6 pi/5) L0^(5/3).
    The lattice reaches 128 f0; the neglected tail is about (f0/f_max)^(5/3) = 3e-4."""
    r0 = 0.07
    for L0 in (1.0, 20.0):
        fm, f0 = osc.psd_scales(0.0, L0)
        assert np.isinf(fm) and f0 == pytest.approx(1.0 / L0)
        df = f0 / 8
        w = osc.mvk_psd(_lattice_f2(2048, df), r0, fm, f0)
        var = w.sum() * df * df
        closed = 0.023 * r0 ** (-5.0 / 3.0) * (6.0 * np.pi / 5.0) * L0 ** (5.0 / 3.0)
        assert var / closed - 1 == pytest.approx(0.0, abs=1e-3), (L0, var / closed)
        assert var < closed  # only the tail beyond the lattice is missing


@pytest.mark.parametrize("alpha", [11.0 / 3.0, 4.35, 3.3])
@pytest.mark.parametrize("l0,L0,conv", [(0.05, 1.0, 0), (0.05, 1.5, 1), (0.2, 0.5, 0)])
def test_psd_variance_and_gradient_confluent_closed_forms(alpha, l0, L0, conv):
    r0 = 0.05
    fm, f0 = osc.psd_scales(l0, L0, conv)
    c = f0 * f0
    df = f0 / 6
    n = 2048
    assert (n // 2) * df > 6 * fm  # exp(-36) of the Gaussian cut-off left beyond the lattice
    f2 = _lattice_f2(n, df)
    w = osc.mvk_psd(f2, r0, fm, f0, alpha)
    var = w.sum() * df * df
    grad = (4 * np.pi ** 2 * f2 * w).sum() * df * df
    a = 0.023 * r0 ** (-5.0 / 3.0)
    var_closed = a * np.pi * c ** (1 - alpha / 2) * sp.hyperu(1.0, 2 - alpha / 2, c / fm ** 2)
    grad_closed = a * 4 * np.pi ** 3 * c ** (2 - alpha / 2) * sp.hyperu(2.0, 3 - alpha / 2, c / fm ** 2)
    assert var / var_closed - 1 == pytest.approx(0.0, abs=1e-9)
    assert grad / grad_closed - 1 == pytest.approx(0.0, abs=1e-9)


def test_inner_scale_conventions_in_rad_per_metre():
    """The Gaussian factor of Eq. S17 is exp(-kappa^2/kappa_m^2) with kappa in
    rad/m: kappa_m = 2 pi / l0 as printed, 5.92 / l0 with inner_scale_conv = 1."""
    l0, L0, r0 = 0.004, 10.0, 0.1
    kappa = np.array([50.0, 400.0, 1480.0, 3000.0])  # rad/m
    f2 = (kappa / (2 * np.pi)) ** 2                    # cycles/m, squared
    for conv, kappa_m in ((0, 2 * np.pi / l0), (1, 5.92 / l0)):
        fm, f0 = osc.psd_scales(l0, L0, conv)
        ratio = osc.mvk_psd(f2, r0, fm, f0) / osc.mvk_psd(f2, r0, np.inf, f0)
        assert np.allclose(ratio, np.exp(-(kappa / kappa_m) ** 2), rtol=1e-12, atol=0)


def _r2_mean(u, dx):
    n = u.shape[-1]
    x = (np.arange(n) - n // 2) * dx
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    i = np.abs(u) ** 2
    return (i * r2).sum(axis=(-1, -2)) / i.sum(axis=(-1, -2))


def test_beam_second_moment_invariant():
    """E<r^2> - <r^2>_vac against sum_i (L - z_i)^2 E|grad phi_i|^2 / k^2.

    Unequal screen strengths make the (L - z_i)^2 weighting differ from the
    z_i^2 of the reversed path by a factor of about 4; the inner scale
    (l0 = 2 cm, fm = 50 cycles/m against the 128 cycles/m Nyquist frequency)
    keeps the phase gradient resolved and the beam stays far from the edges."""
    n, side, lam, length = 256, 1.0, 1.55e-6, 2000.0
    weights = np.array([3.0, 1.0, 1.0, 0.2])
    m = len(weights)
    cn2dz = tuple(1e-14 * (length / m) * weights)
    dz = tuple([length / (2 * m)] + [length / m] * (m - 1) + [length / (2 * m)])
    p = workloads.Path(n=n, dx=side / n, wavelength=lam, dz=dz, cn2dz=cn2dz, l0=0.02, L0=0.5,
                       realizations=160)
    u0 = workloads.gaussian_source(n, p.dx, 0.05)
    phi = osc.phase_screens(p, seed=31)
    u, _ = opr.propagate(u0, p, phi)
    uv, _ = opr.propagate(u0, p.with_(realizations=1), np.zeros((1, m, n, n)))
    d = _r2_mean(u, p.dx) - _r2_mean(uv, p.dx)[0]

    k = 2 * np.pi * p.n0 / lam
    df = 1.0 / (n * p.dx)
    f2 = _lattice_f2(n, df)
    fm, f0 = osc.psd_scales(p.l0, p.L0)
    z = np.cumsum(dz)[:-1]
    expect, reversed_path = 0.0, 0.0
    for i in range(m):
        r0 = osc.fried_parameter(lam, p.n0, cn2dz[i])
        w = osc.mvk_psd(np.where(f2 > 0, f2, 1.0), r0, fm, f0)
        w[0, 0] = 0.0
        g2 = (4 * np.pi ** 2 * f2 * w).sum() * df * df
        expect += (length - z[i]) ** 2 * g2 / k ** 2
        reversed_path += z[i] ** 2 * g2 / k ** 2
    se = d.std(ddof=1) / np.sqrt(len(d))
    assert abs(d.mean() - expect) < 4 * se, (d.mean(), expect, se)
    assert se < 0.1 * expect
    assert abs(d.mean() - reversed_path) > 8 * se  # the test tells the two weightings apart
