"""Ensemble moments taken inside the forward pass (Sec. 3.3): a plan bound to
a Moments buffer adds every forward call's output fields to it, inside the
final inverse row transform where the pass ends with one.  The sums must be
those of a separate moment pass over the call's output bit for bit, over
chunk layouts with empty, uneven and multi-row chunks; the output equals an
unbound plan's to within rounding (its final transform runs in another
kernel, whose multiply-adds the compiler may fuse differently); the
finalized statistics must match the FP64 oracle's."""
import numpy as np
import pytest
import torch

from oracle import stats as ost
from paper_2604_07248_amd import workloads

from gpu_helpers import oracle_propagate, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_2604_07248_amd import api as _api
    return _api


def c64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def _path(n, r, case):
    lam = 1e-6
    dx = 2e-3 if n >= 128 else 4e-3
    limit = n * dx * dx / lam
    if case in ("no_screens", "no_screens_no_distance"):
        dz = (0.5 * limit,) if case == "no_screens" else (0.0,)
        return workloads.Path(n=n, dx=dx, wavelength=lam, dz=dz, cn2dz=(), realizations=r)
    base = workloads.uniform_path(n, n * dx, lam, min(2.4 * limit, 2000.0), 3, 1e-15, 0.005, 20.0,
                                  3 if case == "sh" else 0, realizations=r)
    if case == "last_zero":
        return base.with_(dz=base.dz[:-1] + (0.0,))
    return base


def _source(path, shared):
    u0 = workloads.gaussian_source(path.n, path.dx, 0.1 * path.n * path.dx)
    if shared:
        return c64(u0)
    rng = np.random.default_rng(path.n + path.realizations)
    amp = 1 + 0.1 * rng.standard_normal((path.realizations, path.n, path.n))
    return c64(u0[None] * amp)


# (n, realizations, case, shared source): moment_chunks(n) is 64 at n = 16,
# 16 at 256 and 4 from 1024, so these cover chunks that are all empty but
# some, uneven chunks, several realizations per chunk and one per chunk; the
# last four take the fallback (a screen at the receiver plane, or no
# transform at all) or a shared source read with stride 0.
CASES = [
    (16, 3, "plain", False),
    (64, 5, "plain", True),
    (256, 64, "plain", False),
    (512, 1, "plain", True),
    (1024, 9, "sh", False),
    (1024, 64, "plain", True),
    (2048, 5, "plain", False),
    (128, 5, "last_zero", False),
    (128, 6, "no_screens", True),
    (128, 4, "no_screens_no_distance", False),
]


@pytest.mark.parametrize("n,r,case,shared", CASES)
def test_fused_moments_bitwise(api, n, r, case, shared):
    path = _path(n, r, case)
    say(f"[moments] n={n} R={r} case={case} shared={shared}")
    fused, plain = api.Plan(path), api.Plan(path)
    mf, mp = api.Moments(n, path.dx), api.Moments(n, path.dx)
    fused.bind_moments(mf)
    u = _source(path, shared)
    for seed in (3, 4):  # the second call adds to non-zero sums
        a = fused.propagate(u, seed=seed)
        b = plain.propagate(u, seed=seed)
        assert float((a - b).abs().max()) <= 1e-6 * float(b.abs().max())
        mp.add(a)
    torch.cuda.synchronize()
    assert mf.count == mp.count == 2 * r
    assert torch.equal(mf.buf, mp.buf)
    fused.bind_moments(None)
    before = mf.buf.clone()
    fused.propagate(u, seed=5)
    torch.cuda.synchronize()
    assert torch.equal(mf.buf, before) and mf.count == 2 * r


def test_fused_moments_ar_step(api):
    path = _path(256, 6, "sh")
    say("[moments] AR step n=256 R=6")
    fused, plain = api.Plan(path), api.Plan(path)
    sf, sp = fused.init_spectra(21), plain.init_spectra(21)
    mf, mp = api.Moments(path.n, path.dx), api.Moments(path.n, path.dx)
    fused.bind_moments(mf)
    u = _source(path, True)
    for t in (1, 2):
        a = fused.evolve_propagate(sf, 21, t, 0.95, 0.4, -0.25, u_in=u)
        b = plain.evolve_propagate(sp, 21, t, 0.95, 0.4, -0.25, u_in=u)
        assert float((a - b).abs().max()) <= 1e-6 * float(b.abs().max())
        mp.add(a)
    torch.cuda.synchronize()
    assert torch.equal(mf.buf, mp.buf) and mf.count == 2 * path.realizations


def test_fused_moments_match_oracle(api):
    w = workloads.config1()
    say("[moments] config 1 against the oracle")
    u0 = w.source_field().astype(np.complex64)
    plan = api.Plan(w.path)
    m = api.Moments(w.path.n, w.path.dx)
    plan.bind_moments(m)
    plan.propagate(c64(u0), seed=w.seed)
    _, s = m.finalize()
    ref, _ = oracle_propagate(w.path, w.seed, u0)
    so = ost.summary(ref, w.path.dx)
    assert s["count"] == w.path.realizations
    for key, tol in (("si_plane", 1e-3), ("w_2nd", 1e-4), ("w_fit", 1e-2)):
        assert abs(s[key] - so[key]) <= tol * abs(so[key]), (key, s[key], so[key])


def test_bind_moments_checks_shape(api):
    path = _path(64, 2, "plain")
    plan = api.Plan(path)
    with pytest.raises(ValueError):
        plan.bind_moments(api.Moments(128, path.dx))
