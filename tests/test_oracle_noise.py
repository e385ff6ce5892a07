"""Pins for the oracle's counter-based generator and Gaussian noise."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats as sps

from oracle import noise, philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available for the independent Philox reference")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", os.path.join(HERE, "philox_ref.cpp"),
                    "-o", exe], check=True, capture_output=True)

    def run(key, ctrs):
        text = f"{key[0]} {key[1]}\n" + "\n".join(" ".join(str(int(c)) for c in row) for row in ctrs)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(w, 16) for w in line.split()] for line in out.strip().splitlines()], dtype=np.uint32)
    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_bit_exact_vs_rocrand(rocrand_philox):
    rng = np.random.default_rng(123)
    ctrs = rng.integers(0, 2 ** 32, size=(2000, 4), dtype=np.uint64)
    ctrs[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 0, 1 << 31]]
    for key in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (12345, 678), (0xDEADBEEF, 0x01234567)]:
        ours = philox.philox4x32_10(ctrs, key)
        ref = rocrand_philox(key, ctrs)
        assert np.array_equal(ours, ref), f"key {key}: {np.sum(ours != ref)} words differ"


def test_philox_layout_counters_vs_rocrand(rocrand_philox):
    # the counters the main-spectrum and subharmonic draws use
    n = 64
    e = np.arange(n // 2 * n, dtype=np.uint64)
    ctrs = noise.counters(e, 7, 5, noise.TAG_MAIN, 3).reshape(-1, 4)
    key = noise.seed_key(0x123456789)
    assert np.array_equal(philox.philox4x32_10(ctrs, key), rocrand_philox(key, ctrs))


def test_uniform_map_endpoints():
    u = noise.uniform_open01(np.array([0, 511, 512, 0xFFFFFFFF], dtype=np.uint64))
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)  # exact in FP32


def test_box_muller_moments_and_normality():
    z = noise.spectral_noise(512, seed=99, t=0, pair=0, screen=0)
    x = np.concatenate([z.real.ravel(), z.imag.ravel()])
    n = x.size
    assert abs(x.mean()) < 4.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 4.0 * np.sqrt(2.0 / n)
    assert abs(np.mean(z.real * z.imag)) < 4.0 / np.sqrt(z.size)
    assert sps.kstest(x[:200000], "norm").pvalue > 1e-4
    # real and imaginary parts each unit variance (Parseval reading of N_c)
    assert abs(z.real.var() - 1.0) < 4.0 * np.sqrt(2.0 / z.size)


def test_noise_streams_distinct():
    a = noise.spectral_noise(32, 1, 0, 0, 0)
    for args in [(2, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (1, 0, 0, 1)]:
        b = noise.spectral_noise(32, *args)
        assert abs(np.corrcoef(a.real.ravel(), b.real.ravel())[0, 1]) < 0.1
    c = noise.spectral_noise(32, 1, 0, 0, 0, tag=noise.TAG_AR)
    assert not np.allclose(a, c)
    assert np.array_equal(a, noise.spectral_noise(32, 1, 0, 0, 0))


def test_subharmonic_noise_layout():
    sh = noise.subharmonic_noise(3, seed=4, t=0, pair=2, screen=1)
    assert sh.shape == (3, 8)
    v = philox.philox4x32_10(noise.counters(np.array([5], dtype=np.uint64), 0, 2, noise.TAG_SH, 1),
                             noise.seed_key(4))[0]
    # level 2, offsets q = 2 and 3 come from counter e = 4 + 1
    assert np.isclose(sh[1, 2], noise.box_muller(v[0], v[1]))
    assert np.isclose(sh[1, 3], noise.box_muller(v[2], v[3]))
