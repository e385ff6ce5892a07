"""Seeded synthetic workloads: path geometries, source fields and seeds.

This module is the one place that both the FP64 oracle (through the tests) and
the GPU path take their inputs from.  It holds none of the method's arithmetic:
only geometry (grid, step lengths, integrated Cn^2 per interval), the source
fields, seeds and the workload catalogue.

The workloads are shaped like the paper's experiments, with uniform-Cn^2 paths
standing in for its Hufnagel-Valley profiles: collimated Gaussian beams or
plane waves, modified von Karman turbulence with inner/outer scales, one screen
at the midpoint of each of M equal intervals (distances
[L/2M, L/M, ..., L/M, L/2M]), integrated strength Cn^2 * L / M per screen.
"""

from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np

TF_FRESNEL = 0
TF_ANGULAR_SPECTRUM = 1


@dataclass(frozen=True)
class Path:
    """One propagation path; mirrors the C struct turpy_path."""
    n: int
    dx: float
    wavelength: float
    dz: Tuple[float, ...]          # M + 1 diffraction distances [m]
    cn2dz: Tuple[float, ...]       # M integrated Cn^2 values [m^(1/3)]
    l0: float = 0.0                # inner scale [m]; 0 disables the cutoff
    L0: float = float("inf")       # outer scale [m]; inf disables it
    sh_levels: int = 0             # subharmonic levels (0..3)
    n0: float = 1.0                # mean refractive index
    tf_kind: int = TF_FRESNEL
    inner_scale_conv: int = 0      # 0: fm = 1/l0, 1: fm = 5.92/(2 pi l0)
    realizations: int = 1
    psd_alpha: float = 0.0         # PSD power law (0: 11/3, the modified von Karman law)

    @property
    def num_screens(self):
        return len(self.cn2dz)

    @property
    def length(self):
        return float(sum(self.dz))

    def with_(self, **kw):
        return replace(self, **kw)


def uniform_path(n, side, wavelength, length, screens, cn2, l0, L0, sh_levels=0,
                 realizations=1, placement="mid", tf_kind=TF_FRESNEL, n0=1.0):
    """Uniform-Cn^2 path with M screens.

    placement "mid": each screen at the middle of its interval,
    dz = [L/2M, L/M x (M-1), L/2M]; "end": dz = [L/M x M, 0].
    """
    step = length / screens
    if placement == "mid":
        dz = (0.5 * step,) + (step,) * (screens - 1) + (0.5 * step,)
    else:
        dz = (step,) * screens + (0.0,)
    return Path(n=n, dx=side / n, wavelength=wavelength, dz=dz,
                cn2dz=(cn2 * step,) * screens, l0=l0, L0=L0, sh_levels=sh_levels,
                n0=n0, tf_kind=tf_kind, realizations=realizations)


def grid(n, dx):
    """Centred coordinates x_i = (i - N/2) dx."""
    return (np.arange(n) - n // 2) * dx


def gaussian_source(n, dx, w0):
    """Collimated Gaussian field exp(-(x^2 + y^2)/W0^2), complex128 [N][N]."""
    x = grid(n, dx)
    return np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / (w0 * w0)).astype(np.complex128)


def plane_wave(n):
    return np.ones((n, n), dtype=np.complex128)


def flat_top(n, dx, width, order=10):
    """Tapered plane wave exp(-(r/width)^(2 order)): flat over the centre of the
    grid and zero at its edge, so that the periodic grid's wrap-around (where
    the non-periodic subharmonic screens jump) carries no field."""
    x = grid(n, dx)
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    return np.exp(-(r2 / (width * width)) ** order).astype(np.complex128)


def seeded_field(shape, seed):
    """Random complex64 field (standard normal components) for adjoint/gradient tests."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def seeded_phase(shape, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(shape)).astype(np.float32)


@dataclass(frozen=True)
class Workload:
    name: str
    path: Path
    seed: int
    source: str = "gaussian"       # "gaussian" | "plane" | "flat_top"
    w0: float = 0.0
    extra: dict = field(default_factory=dict)

    def source_field(self):
        if self.source == "plane":
            return plane_wave(self.path.n)
        if self.source == "flat_top":
            return flat_top(self.path.n, self.path.dx, 0.42 * self.path.n * self.path.dx)
        return gaussian_source(self.path.n, self.path.dx, self.w0)


def config1():
    """Plain forward, N=128 over 0.5 m, 1550 nm, 1 km, 5 screens, Cn2=1e-14,
    l0=1 cm, L0=10 m, no subharmonics, 16 realizations, seed 0, W0=2 cm."""
    p = uniform_path(128, 0.5, 1550e-9, 1000.0, 5, 1e-14, 0.01, 10.0, 0, realizations=16)
    return Workload("c1_n128_m5_r16", p, seed=0, source="gaussian", w0=0.02)


def config2(cn2=1e-15, source="flat_top", realizations=256, seed=20):
    """Weak-to-strong sweep point: N=512 over 1 m, 1550 nm, 2 km, 10 screens with
    3-level subharmonics, l0=5 mm, L0=20 m; plane wave (tapered flat top, see
    flat_top) or W0=3 cm Gaussian."""
    p = uniform_path(512, 1.0, 1550e-9, 2000.0, 10, cn2, 0.005, 20.0, 3, realizations=realizations)
    return Workload(f"c2_n512_m10_cn2_{cn2:g}_{source}", p, seed=seed, source=source, w0=0.03)


def config3(realizations=32, steps=1000):
    """AR temporal evolution: N=1024 over 1 m, 1064 nm, 1.5 km, 8 screens,
    Cn2=2e-14, l0=5 mm, L0=20 m, alpha=0.99, frozen-flow shift (0.5, 0) px/step,
    32 sequences, W0=5 cm Gaussian, seed 3."""
    p = uniform_path(1024, 1.0, 1064e-9, 1500.0, 8, 2e-14, 0.005, 20.0, 0, realizations=realizations)
    return Workload("c3_n1024_m8_ar", p, seed=3, source="gaussian", w0=0.05,
                    extra={"alpha": 0.99, "shift_x": 0.5, "shift_y": 0.0, "steps": steps})


def config4(batch=64):
    """Differentiable path: N=512 over 1 m, 1550 nm, 1 km, 6 screens, Cn2=5e-15,
    l0=5 mm, L0=20 m, batch 64, W0=2 cm, seed 4; two 512x512 masks."""
    p = uniform_path(512, 1.0, 1550e-9, 1000.0, 6, 5e-15, 0.005, 20.0, 0, realizations=batch)
    return Workload("c4_n512_m6_d2nn", p, seed=4, source="gaussian", w0=0.02)


def headline(realizations=64):
    """Headline propagation workload: N=1024 over 1 m, 1064 nm, 1.5 km, 8 fresh
    screens per realization (Cn2=2e-14, l0=5 mm, L0=20 m, no subharmonics),
    64 realizations, W0=5 cm, seed 1."""
    p = uniform_path(1024, 1.0, 1064e-9, 1500.0, 8, 2e-14, 0.005, 20.0, 0, realizations=realizations)
    return Workload("h1_n1024_m8_r64", p, seed=1, source="gaussian", w0=0.05)


def uneven_batch(instances=4096, seed=5):
    """Serving-style mix: N in {256,512,1024,2048}, lambda in {532,1064,1550} nm,
    5-20 screens, log10 Cn2 ~ U[-16,-13], L ~ U[500,5000] m, dx chosen at the
    sampling limit sqrt(2 lambda dz / N), W0 = N dx / 8, 3-level subharmonics,
    one realization per instance.  Drawn with numpy's PCG64 from `seed`."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(instances):
        n = int(rng.choice([256, 512, 1024, 2048]))
        lam = float(rng.choice([532e-9, 1064e-9, 1550e-9]))
        m = int(rng.integers(5, 21))
        cn2 = 10.0 ** rng.uniform(-16, -13)
        length = float(rng.uniform(500.0, 5000.0))
        dz = length / m
        dx = float(np.sqrt(2.0 * lam * dz / n))
        p = uniform_path(n, n * dx, lam, length, m, cn2, 0.005, 20.0, 3, realizations=1)
        out.append(Workload(f"c5_{n}", p, seed=seed, source="gaussian", w0=n * dx / 8))
    return out
