"""Pins for the oracle's dual-domain receiver (Sec. 2.5, Sec. 4.1)."""
import numpy as np

from oracle import receiver


def test_zero_masks_is_aperture_identity():
    rng = np.random.default_rng(0)
    n, dx = 64, 0.01
    u = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    out = receiver.forward(u, np.zeros((n, n)), np.zeros((n, n)), dx)
    assert np.allclose(out, receiver.aperture(n, dx) * u, atol=1e-12)
    a = receiver.aperture(n, dx)
    # 12-inch disc: area within one ring of pixels of pi D^2 / 4
    assert abs(a.sum() * dx * dx - np.pi * 0.3048 ** 2 / 4) < np.pi * 0.3048 * dx * 1.5


def test_receiver_is_unitary_on_the_aperture():
    rng = np.random.default_rng(1)
    n, dx = 32, 0.02
    u = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    t1, t2 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    out = receiver.forward(u, t1, t2, dx)
    a = receiver.aperture(n, dx)
    assert np.allclose(np.sum(np.abs(out) ** 2), np.sum(np.abs(a * u) ** 2), rtol=1e-12)


def test_receiver_adjoint_matches_finite_differences():
    rng = np.random.default_rng(2)
    n, dx = 32, 0.015
    u = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    t1, t2 = 0.3 * rng.standard_normal((n, n)), 0.3 * rng.standard_normal((n, n))
    wgt = rng.random((n, n))

    def loss(uu, a, b):
        return float(np.sum(wgt * np.abs(receiver.forward(uu, a, b, dx)) ** 2))

    out = receiver.forward(u, t1, t2, dx)
    g_u, d1, d2 = receiver.adjoint(2 * wgt * out, u, t1, t2, dx)
    h = 1e-6
    for (i, j) in [(16, 16), (12, 19), (20, 9)]:
        e = np.zeros((n, n)); e[i, j] = h
        fd1 = (loss(u, t1 + e, t2) - loss(u, t1 - e, t2)) / (2 * h)
        fd2 = (loss(u, t1, t2 + e) - loss(u, t1, t2 - e)) / (2 * h)
        assert abs(fd1 - d1[i, j]) < 1e-7 * max(1, abs(fd1))
        assert abs(fd2 - d2[i, j]) < 1e-7 * max(1, abs(fd2))
        du = np.zeros((3, n, n), dtype=complex); du[1, i, j] = h
        fdu = (loss(u + du, t1, t2) - loss(u - du, t1, t2)) / (2 * h)
        assert abs(fdu - g_u[1, i, j].real) < 1e-7 * max(1, abs(fdu))
