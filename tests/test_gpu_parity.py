"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by
element on the same seeded inputs (field relative-L2 <= 1e-4 in complex64)."""
import numpy as np
import pytest
import torch

from oracle import evolve as oev
from oracle import propagate as opr
from oracle import stats as ost
from paper_2604_07248_amd import workloads

from gpu_helpers import TOL, oracle_propagate, oracle_screens, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_2604_07248_amd import api as _api
    return _api


def c64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def sized_path(n, realizations=3, m=2, sh=0, **kw):
    """A path on an N-point grid whose steps sit below the sampling limit."""
    lam = 1e-6
    dx = 2e-3 if n >= 128 else 4e-3
    limit = n * dx * dx / lam
    length = min(0.8 * limit * m, 2000.0) if m > 0 else 0.5 * limit
    side = n * dx
    if m == 0:
        return workloads.Path(n=n, dx=dx, wavelength=lam, dz=(length,), cn2dz=(), l0=0.005, L0=20.0,
                              sh_levels=sh, realizations=realizations, **kw)
    return workloads.uniform_path(n, side, lam, length, m, 1e-15, 0.005, 20.0, sh, realizations=realizations).with_(**kw)


def gaussian(path, w0_frac=0.1):
    return workloads.gaussian_source(path.n, path.dx, w0_frac * path.n * path.dx)


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048])
def test_screens_match_oracle(api, n):
    path = sized_path(n, realizations=3, m=2, sh=3 if n in (64, 512) else 0)
    if n in (128, 1024):
        path = path.with_(psd_alpha=4.35 if n == 128 else 3.3)
    say(f"[screens] n={n} sh={path.sh_levels}")
    plan = api.Plan(path)
    got = plan.screens(seed=7).cpu().numpy()
    ref = oracle_screens(path, 7, range(3))
    err = rel_l2(got, ref)
    say(f"[screens] n={n} rel-L2 {err:.2e}")
    assert err < TOL


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048])
def test_propagate_sizes(api, n):
    path = sized_path(n)
    say(f"[propagate] n={n}")
    u0 = gaussian(path)
    plan = api.Plan(path)
    out, ck = plan.propagate(c64(u0), seed=11, checkpoints=True)
    ref, ref_ck = oracle_propagate(path, 11, u0.astype(np.complex64))
    err = rel_l2(out.cpu().numpy(), ref)
    cerr = rel_l2(ck.cpu().numpy(), ref_ck)
    say(f"[propagate] n={n} field {err:.2e} checkpoints {cerr:.2e}")
    assert err < TOL and cerr < TOL


def test_config1_full(api):
    w = workloads.config1()
    say("[config1] N=128 R=16 M=5")
    u0 = w.source_field().astype(np.complex64)
    plan = api.Plan(w.path)
    out = plan.propagate(c64(u0), seed=w.seed).cpu().numpy()
    ref, _ = oracle_propagate(w.path, w.seed, u0)
    per = [rel_l2(out[r], ref[r]) for r in range(w.path.realizations)]
    say(f"[config1] worst per-realization rel-L2 {max(per):.2e}")
    assert max(per) < TOL
    # statistics of the batch against the oracle's
    m = api.Moments(w.path.n, w.path.dx)
    m.add(torch.from_numpy(out).cuda())
    _, s = m.finalize()
    so = ost.summary(ref, w.path.dx)
    for key, tol in (("si_plane", 1e-3), ("w_2nd", 1e-4), ("w_fit", 1e-2)):
        assert abs(s[key] - so[key]) <= tol * abs(so[key]), (key, s[key], so[key])


@pytest.mark.parametrize("case", ["angular", "first_zero", "last_zero", "no_screens", "per_realization_source",
                                  "subharmonics", "inner_conv", "kolmogorov", "single", "odd_pairs",
                                  "tissue_psd", "ocean_psd"])
def test_propagate_options(api, case):
    path = sized_path(256, realizations=4, m=3)
    if case == "angular":
        path = path.with_(tf_kind=1)
    elif case == "first_zero":
        path = path.with_(dz=(0.0,) + path.dz[1:])
    elif case == "last_zero":
        path = path.with_(dz=path.dz[:-1] + (0.0,))
    elif case == "no_screens":
        path = sized_path(256, realizations=2, m=0)
    elif case == "subharmonics":
        path = path.with_(sh_levels=3)
    elif case == "inner_conv":
        path = path.with_(inner_scale_conv=1)
    elif case == "kolmogorov":
        path = path.with_(l0=0.0, L0=float("inf"), sh_levels=2)
    elif case == "single":
        path = path.with_(realizations=1)
    elif case == "odd_pairs":
        path = path.with_(realizations=5)
    elif case == "tissue_psd":
        path = path.with_(psd_alpha=4.35, sh_levels=3)
    elif case == "ocean_psd":
        path = path.with_(psd_alpha=5.0)
    say(f"[options] {case}")
    u0 = gaussian(path)
    if case == "per_realization_source":
        rng = np.random.default_rng(3)
        u0 = u0[None] * np.exp(1j * 0.3 * rng.standard_normal((path.realizations, path.n, path.n)))
    u0 = u0.astype(np.complex64)
    plan = api.Plan(path)
    out = plan.propagate(c64(u0), seed=5).cpu().numpy()
    ref, _ = oracle_propagate(path, 5, u0)
    err = rel_l2(out, ref)
    say(f"[options] {case} rel-L2 {err:.2e}")
    assert err < TOL


def test_angular_spectrum_evanescent_grid(api):
    """dx = lambda/2: the grid's outer bins have kappa > k and decay
    (evanescent), so the angular-spectrum correction comes from the plan's
    FP64 radial table instead of the FP32 propagating-only form."""
    lam, dx, n = 1e-6, 0.5e-6, 64
    path = workloads.Path(n=n, dx=dx, wavelength=lam, dz=(4e-6, 7e-6, 4e-6), cn2dz=(2e-17, 2e-17),
                          l0=0.0, L0=float("inf"), tf_kind=workloads.TF_ANGULAR_SPECTRUM, realizations=3)
    say("[options] evanescent n=64 dx=lambda/2")
    u0 = workloads.seeded_field((n, n), 13)  # broadband: energy in the evanescent bins too
    plan = api.Plan(path)
    out, ck = plan.propagate(c64(u0), seed=11, checkpoints=True)
    ref, ref_ck = oracle_propagate(path, 11, u0)
    err = rel_l2(out.cpu().numpy(), ref)
    kept = float(np.sum(np.abs(ref[0]) ** 2) / np.sum(np.abs(u0.astype(np.complex128)) ** 2))
    assert kept < 0.9  # the decay of the evanescent bins is part of what is compared
    rng = np.random.default_rng(12)
    g = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)).astype(np.complex64)
    g_in, _ = plan.propagate_backward(c64(g), ck, seed=11)
    phi = oracle_screens(path, 11, range(3))
    ref_gin, _ = opr.propagate_adjoint(g.astype(np.complex128), path, phi, ref_ck)
    eg = rel_l2(g_in.cpu().numpy(), ref_gin)
    say(f"[options] evanescent rel-L2 {err:.2e} grad_in {eg:.2e} energy kept {kept:.3f}")
    assert err < TOL and eg < TOL


def test_materialized_equals_synthesised(api):
    path = sized_path(512, realizations=4, m=3, sh=3)
    say("[materialized] n=512")
    plan = api.Plan(path)
    u0 = c64(gaussian(path))
    phi = plan.screens(seed=9)
    a = plan.propagate(u0, seed=9)
    b = plan.propagate(u0, seed=0, screens=phi)
    err = rel_l2(b.cpu().numpy(), a.cpu().numpy())
    say(f"[materialized] rel diff {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("case", ["synth", "materialized", "angular_edges"])
def test_backward_matches_oracle_adjoint(api, case):
    path = sized_path(256, realizations=3, m=3, sh=3 if case == "synth" else 0)
    if case == "angular_edges":
        path = path.with_(tf_kind=1, dz=(0.0,) + path.dz[1:-1] + (0.0,))
    say(f"[backward] {case}")
    plan = api.Plan(path)
    u0 = gaussian(path).astype(np.complex64)
    rng = np.random.default_rng(4)
    g_out = (rng.standard_normal((3, path.n, path.n)) + 1j * rng.standard_normal((3, path.n, path.n))).astype(np.complex64)
    screens = plan.screens(seed=13) if case != "synth" else None
    out, ck = plan.propagate(c64(u0), seed=13, screens=screens, checkpoints=True)
    g_in, g_phi = plan.propagate_backward(c64(g_out), ck, seed=13, screens=screens)
    phi = oracle_screens(path, 13, range(3))
    ref_out, ref_ck = opr.propagate(u0.astype(np.complex128), path, phi)
    ref_gin, ref_gphi = opr.propagate_adjoint(g_out.astype(np.complex128), path, phi, ref_ck)
    e_in = rel_l2(g_in.cpu().numpy(), ref_gin)
    e_phi = rel_l2(g_phi.cpu().numpy(), ref_gphi)
    say(f"[backward] {case} grad_u_in {e_in:.2e} grad_phi {e_phi:.2e}")
    assert e_in < TOL and e_phi < TOL


def test_evolve_and_spectra_propagation(api):
    path = sized_path(256, realizations=4, m=2)
    say("[evolve] n=256")
    plan = api.Plan(path)
    spec = plan.init_spectra(seed=3)
    ref = oev.initial_spectra(path, 3)
    assert rel_l2(spec.cpu().numpy(), ref) < TOL
    for t in (1, 2, 3):
        plan.evolve(spec, seed=3, t=t, alpha=0.9, shift_x=0.5, shift_y=-0.25)
        ref = oev.evolve(ref, path, 3, t, 0.9, 0.5, -0.25)
    e_spec = rel_l2(spec.cpu().numpy(), ref)
    u0 = gaussian(path).astype(np.complex64)
    out = plan.propagate(c64(u0), spectra=spec).cpu().numpy()
    phi = oev.screens_from_spectra(ref, path.realizations)
    ref_out, _ = opr.propagate(u0.astype(np.complex128), path, phi)
    e_out = rel_l2(out, ref_out)
    say(f"[evolve] spectra {e_spec:.2e} field {e_out:.2e}")
    assert e_spec < TOL and e_out < TOL


def test_ar_resume_is_exact(api):
    """Resuming an AR sequence (Sec. 2.3) from a copy of its state: the pair
    spectra and the subharmonic coefficients after step k, evolved on in a
    fresh plan, give bit for bit the fields of the uninterrupted run, because
    the noise of every step is keyed by (seed, t) alone."""
    path = sized_path(256, realizations=4, m=2, sh=3)
    say("[resume] n=256 sh=3")
    plan = api.Plan(path)
    spec = plan.init_spectra(seed=5)
    for t in (1, 2):
        plan.evolve(spec, seed=5, t=t, alpha=0.95, shift_x=0.5, shift_y=0.25)
    saved = spec._base.clone()  # the whole state buffer: spectra, then the subharmonic tail
    u0 = c64(gaussian(path))
    outs = []
    for t in (3, 4, 5):
        plan.evolve(spec, seed=5, t=t, alpha=0.95, shift_x=0.5, shift_y=0.25)
        outs.append(plan.propagate(u0, spectra=spec).clone())
    plan.close()
    plan2 = api.Plan(path)
    spec2 = saved[: spec.numel()].view(spec.shape)
    for i, t in enumerate((3, 4, 5)):
        plan2.evolve(spec2, seed=5, t=t, alpha=0.95, shift_x=0.5, shift_y=0.25)
        assert torch.equal(plan2.propagate(u0, spectra=spec2), outs[i]), t
    plan2.close()


def test_evolve_with_subharmonics(api):
    """AR state with three subharmonic levels: at t = 0 it reproduces the
    synthesised screens; after three Eq. 4 + Eq. 5 steps (fractional shifts)
    the spectra, the subharmonic coefficients, the propagated field and the
    adjoint match the oracle."""
    path = sized_path(256, realizations=3, m=2, sh=3)
    say("[evolve-sh] n=256 sh=3")
    plan = api.Plan(path)
    u0 = gaussian(path).astype(np.complex64)
    spec = plan.init_spectra(seed=4)
    ref_c, ref_d = oev.initial_spectra(path, 4), oev.initial_sh(path, 4)
    sh = plan.sh_coefficients(spec)
    assert rel_l2(sh[:, :, :24].cpu().numpy(), ref_d.reshape(ref_d.shape[0], ref_d.shape[1], 24)) < TOL
    a = plan.propagate(c64(u0), spectra=spec).cpu().numpy()
    b = plan.propagate(c64(u0), seed=4).cpu().numpy()  # the synthesised screens of t = 0
    e0 = rel_l2(a, b)
    for t in (1, 2, 3):
        plan.evolve(spec, seed=4, t=t, alpha=0.9, shift_x=0.6, shift_y=-0.35)
        ref_c = oev.evolve(ref_c, path, 4, t, 0.9, 0.6, -0.35)
        ref_d = oev.evolve_sh(ref_d, path, 4, t, 0.9, 0.6, -0.35)
    e_spec = rel_l2(spec.cpu().numpy(), ref_c)
    e_sh = rel_l2(sh[:, :, :24].cpu().numpy(), ref_d.reshape(ref_d.shape[0], ref_d.shape[1], 24))
    out, ck = plan.propagate(c64(u0), spectra=spec, checkpoints=True)
    phi = oev.screens_from_state(ref_c, ref_d, path, path.realizations)
    ref_out, ref_ck = opr.propagate(u0.astype(np.complex128), path, phi)
    e_out = rel_l2(out.cpu().numpy(), ref_out)
    rng = np.random.default_rng(5)
    g = (rng.standard_normal(ref_out.shape) + 1j * rng.standard_normal(ref_out.shape)).astype(np.complex64)
    g_in, g_phi = plan.propagate_backward(c64(g), ck, spectra=spec)
    ref_gin, ref_gphi = opr.propagate_adjoint(g.astype(np.complex128), path, phi, ref_ck)
    e_gin, e_gphi = rel_l2(g_in.cpu().numpy(), ref_gin), rel_l2(g_phi.cpu().numpy(), ref_gphi)
    say(f"[evolve-sh] t=0 state vs synthesised {e0:.2e}; spectra {e_spec:.2e} sh {e_sh:.2e} field {e_out:.2e} "
        f"grad_in {e_gin:.2e} grad_phi {e_gphi:.2e}")
    assert e0 < 1e-5 and e_spec < TOL and e_sh < TOL and e_out < TOL and e_gin < TOL and e_gphi < TOL
    with pytest.raises(ValueError):
        plan.propagate(c64(u0), spectra=spec.clone())  # a copy without the subharmonic block


def test_stats_match_oracle(api):
    rng = np.random.default_rng(8)
    n, dx = 128, 0.004
    # a wide beam: FP32 moments hold I^2 only above ~1e-38 (the FP64 oracle has no such floor)
    u = workloads.gaussian_source(n, dx, 0.15)[None] * (1 + 0.3 * rng.standard_normal((40, n, n)))
    u = u.astype(np.complex64)
    m = api.Moments(n, dx)
    m.add(torch.from_numpy(u[:25]).cuda())
    m.add(torch.from_numpy(u[25:]).cuda())
    si, s = m.finalize()
    so = ost.summary(u.astype(np.complex128), dx)
    m1, m2 = ost.moments(u.astype(np.complex128))
    si_ref = ost.si_map(m1, m2)
    assert s["count"] == 40
    assert np.max(np.abs(si.cpu().numpy() - si_ref)) < 1e-4 * np.max(np.abs(si_ref)) + 1e-5
    for key in ("si_plane", "w_2nd", "w_fit"):
        assert abs(s[key] - so[key]) <= 1e-4 * abs(so[key]), (key, s[key], so[key])


_UNEVEN = []


@pytest.mark.parametrize("n", [256, 512, 1024, 2048])
def test_uneven_batch_instances(api, n):
    """Serving-mix instances (one realization each, three subharmonic levels,
    dx at the sampling limit sqrt(2 lambda dz / N)): at each grid size the
    first instance with the fewest screens.  The Fresnel phase at the grid
    corner reaches pi N / 4 rad (1608 rad at N = 2048), so the chirp tables
    rely on their FP64 range reduction."""
    if not _UNEVEN:
        _UNEVEN.extend(workloads.uneven_batch())
    w = min((x for x in _UNEVEN if x.path.n == n), key=lambda x: x.path.num_screens)
    p = w.path
    corner = np.pi * p.wavelength * max(p.dz) * 2 * (0.5 / p.dx) ** 2
    say(f"[uneven] n={n} M={p.num_screens} lambda={p.wavelength:g} L={p.length:.0f} corner phase {corner:.0f} rad")
    plan = api.Plan(p)
    u0 = w.source_field().astype(np.complex64)
    out = plan.propagate(c64(u0), seed=w.seed).cpu().numpy()
    ref, _ = oracle_propagate(p, w.seed, u0)
    err = rel_l2(out, ref)
    say(f"[uneven] n={n} rel-L2 {err:.2e}")
    assert err < TOL


def test_determinism(api):
    path = sized_path(512, realizations=4, m=3, sh=3)
    plan = api.Plan(path)
    u0 = c64(gaussian(path))
    a = plan.propagate(u0, seed=21).cpu().numpy()
    b = plan.propagate(u0, seed=21).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_headline_full_size_sampled(api):
    """Full headline workload (N=1024, R=64, M=8) in the benchmark's launch
    configuration; sampled realizations checked one by one against the oracle:
    the forward fields, and the gradients of the checkpointed and of the
    checkpoint-free adjoint."""
    w = workloads.headline()
    say("[headline] N=1024 R=64 M=8")
    plan = api.Plan(w.path)
    u0 = w.source_field().astype(np.complex64)
    out_t, ck = plan.propagate(c64(u0), seed=w.seed, checkpoints=True)
    g = torch.ones_like(out_t) * (1.0 / 1024)
    g_in, g_phi = plan.propagate_backward(g, ck, seed=w.seed)
    del ck
    # the checkpoint-free adjoint, rebuilding the screen-plane fields from the output
    r_in, r_phi = plan.propagate_backward(g, None, seed=w.seed, u_out=out_t)
    out = out_t.cpu().numpy()
    sample = [0, 1, 37, 63]
    phi = oracle_screens(w.path, w.seed, sample)
    ref, ref_ck = opr.propagate(u0.astype(np.complex128), w.path, phi)
    ref_gin, ref_gphi = opr.propagate_adjoint(np.ones_like(ref) / 1024, w.path, phi, ref_ck)
    for i, r in enumerate(sample):
        e = rel_l2(out[r], ref[i])
        eg = rel_l2(g_in[r].cpu().numpy(), ref_gin[i])
        ep = rel_l2(g_phi[r].cpu().numpy(), ref_gphi[i])
        rg = rel_l2(r_in[r].cpu().numpy(), ref_gin[i])
        rp = rel_l2(r_phi[r].cpu().numpy(), ref_gphi[i])
        say(f"[headline] r={r} field {e:.2e} grad_in {eg:.2e} grad_phi {ep:.2e}; "
            f"checkpoint-free grad_in {rg:.2e} grad_phi {rp:.2e}")
        assert e < TOL and eg < TOL and ep < TOL and rg < TOL and rp < TOL
    # energy is conserved by every realization (unitary steps)
    e0 = np.sum(np.abs(u0.astype(np.complex128)) ** 2)
    assert np.max(np.abs(np.sum(np.abs(out.astype(np.complex128)) ** 2, axis=(1, 2)) / e0 - 1)) < 1e-4


@pytest.mark.parametrize("cn2,source", [(1e-14, "gaussian"), (5e-14, "flat_top")])
def test_config2_full_size_sampled(api, cn2, source):
    """Config 2 at full size (N = 512, 256 realizations, 10 screens with
    3-level subharmonics) at its middle and strongest points, in the tuned
    launch configuration: forward and adjoint, sampled realizations (both of
    the first pair, one inside, the last) against the oracle one by one."""
    w = workloads.config2(cn2=cn2, source=source, seed=30)
    say(f"[config2 full] N=512 R=256 M=10 sh=3 cn2={cn2:g} {source}")
    plan = api.Plan(w.path)
    plan.tune()
    u0 = w.source_field().astype(np.complex64)
    out, ck = plan.propagate(c64(u0), seed=w.seed, checkpoints=True)
    g = torch.ones_like(out) * (1.0 / 512)
    g_in, g_phi = plan.propagate_backward(g, ck, seed=w.seed)
    out = out.cpu().numpy()
    sample = [0, 1, 130, 255]
    phi = oracle_screens(w.path, w.seed, sample)
    ref, ref_ck = opr.propagate(u0.astype(np.complex128), w.path, phi)
    ref_gin, ref_gphi = opr.propagate_adjoint(np.ones_like(ref) / 512, w.path, phi, ref_ck)
    for i, r in enumerate(sample):
        e = rel_l2(out[r], ref[i])
        eg = rel_l2(g_in[r].cpu().numpy(), ref_gin[i])
        ep = rel_l2(g_phi[r].cpu().numpy(), ref_gphi[i])
        say(f"[config2 full] r={r} field {e:.2e} grad_in {eg:.2e} grad_phi {ep:.2e}")
        assert e < TOL and eg < TOL and ep < TOL


def test_headline_angular_spectrum_sampled(api):
    """The headline workload with the angular-spectrum transfer function (the
    benchmark's fwd_angular_spectrum leg): sampled realizations against the
    oracle one by one."""
    w = workloads.headline()
    path = w.path.with_(tf_kind=workloads.TF_ANGULAR_SPECTRUM)
    say("[headline as] N=1024 R=64 M=8 angular spectrum")
    plan = api.Plan(path)
    u0 = w.source_field().astype(np.complex64)
    out = plan.propagate(c64(u0), seed=w.seed).cpu().numpy()
    sample = [0, 33, 63]
    ref, _ = opr.propagate(u0.astype(np.complex128), path, oracle_screens(path, w.seed, sample))
    for i, r in enumerate(sample):
        e = rel_l2(out[r], ref[i])
        say(f"[headline as] r={r} field {e:.2e}")
        assert e < TOL


def test_library_loaded_by_host_call_before_gpu_work():
    """A host-only call (screen placement) may load the library before any GPU
    work; plans created afterwards must still find the device.  Run in a fresh
    process so that nothing else has initialised the GPU first."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "from paper_2604_07248_amd import placement\n"
        "p = placement.placed_path(placement.hufnagel_valley(), 1000.0, 1.55e-6, 128, 4e-3, 0.1, realizations=2)\n"
        "import torch\n"
        "from paper_2604_07248_amd import api\n"
        "u0 = torch.ones((128, 128), dtype=torch.complex64, device='cuda')\n"
        "out = api.Plan(p).propagate(u0, seed=1)\n"
        "torch.cuda.synchronize()\n"
        "print('ok', p.num_screens, float(out.abs().square().sum()))\n")
    say("[order] placement before GPU work, fresh process")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=240)
    say(r.stdout.strip(), r.stderr.strip()[-500:])
    assert r.returncode == 0 and r.stdout.startswith("ok")


@pytest.mark.parametrize("case", ["synth", "materialized", "spectra", "angular_edges", "first_zero", "long"])
def test_reversible_backward(api, case):
    """The checkpoint-free adjoint rebuilds the screen-plane fields from the
    forward output (every step is unitary); its gradients equal the
    checkpointed adjoint's up to FP32 rounding and the oracle's to 1e-4."""
    r = 3
    path = sized_path(256, realizations=r, m=3, sh=3 if case in ("synth", "spectra") else 0)
    if case == "angular_edges":
        path = path.with_(tf_kind=1, dz=(0.0,) + path.dz[1:-1] + (0.0,))
    elif case == "first_zero":
        path = path.with_(dz=(0.0,) + path.dz[1:])
    elif case == "long":
        path = sized_path(512, realizations=4, m=8)
        r = 4
    say(f"[reversible] {case} n={path.n} M={path.num_screens}")
    plan = api.Plan(path)
    u0 = gaussian(path).astype(np.complex64)
    rng = np.random.default_rng(6)
    g = (rng.standard_normal((r, path.n, path.n)) + 1j * rng.standard_normal((r, path.n, path.n))).astype(np.complex64)
    kw = {}
    if case == "materialized":
        kw["screens"] = plan.screens(seed=17)
    elif case == "spectra":
        spec = plan.init_spectra(seed=17)
        plan.evolve(spec, seed=17, t=1, alpha=0.95, shift_x=0.4, shift_y=0.2)
        kw["spectra"] = spec
    out, ck = plan.propagate(c64(u0), seed=17, checkpoints=True, **kw)
    a_in, a_phi = plan.propagate_backward(c64(g), ck, seed=17, **kw)
    b_in, b_phi = plan.propagate_backward(c64(g), None, seed=17, u_out=out, **kw)
    d_in = rel_l2(b_in.cpu().numpy(), a_in.cpu().numpy())
    d_phi = rel_l2(b_phi.cpu().numpy(), a_phi.cpu().numpy())
    if case == "spectra":
        phi = oev.screens_from_state(oev.evolve(oev.initial_spectra(path, 17), path, 17, 1, 0.95, 0.4, 0.2),
                                     oev.evolve_sh(oev.initial_sh(path, 17), path, 17, 1, 0.95, 0.4, 0.2), path, r)
    elif case == "materialized":
        phi = kw["screens"].cpu().numpy().astype(np.float64)
    else:
        phi = oracle_screens(path, 17, range(r))
    ref_out, ref_ck = opr.propagate(u0.astype(np.complex128), path, phi)
    ref_in, ref_phi = opr.propagate_adjoint(g.astype(np.complex128), path, phi, ref_ck)
    e_in, e_phi = rel_l2(b_in.cpu().numpy(), ref_in), rel_l2(b_phi.cpu().numpy(), ref_phi)
    say(f"[reversible] {case}: vs checkpointed {d_in:.2e} / {d_phi:.2e}; vs oracle {e_in:.2e} / {e_phi:.2e}")
    assert d_in < 2e-5 and d_phi < 2e-5
    assert e_in < TOL and e_phi < TOL


def test_reversible_autograd_matches_checkpointed(api):
    path = sized_path(128, realizations=2, m=3)
    plan = api.Plan(path)
    u0 = c64(gaussian(path)).requires_grad_(True)
    phi = plan.screens(seed=5).requires_grad_(True)
    grads = []
    for reversible in (False, True):
        out = api.Propagate.apply(u0, phi, plan, 5, 0, reversible)
        loss = (out.abs() ** 2 * torch.linspace(0, 1, path.n, device="cuda")[None, None, :]).sum()
        gu, gp = torch.autograd.grad(loss, (u0, phi))
        grads.append((gu.cpu().numpy(), gp.cpu().numpy()))
    assert rel_l2(grads[1][0], grads[0][0]) < 2e-5 and rel_l2(grads[1][1], grads[0][1]) < 2e-5


def _uneven_sample(count=6, realizations=(1, 2)):
    """Serving-mix instances of every grid size, the cheapest of each."""
    if not _UNEVEN:
        _UNEVEN.extend(workloads.uneven_batch())
    out = []
    for n in (256, 512, 1024, 2048, 256, 512)[:count]:
        cands = sorted((x for x in _UNEVEN if x.path.n == n), key=lambda x: (x.path.num_screens, x.name))
        w = cands[len(out) // 4]
        out.append(w.path.with_(realizations=realizations[len(out) % len(realizations)]))
    return out


def test_uneven_batch_equals_single_plans(api):
    """One batch call over instances of N = 256..2048 with their own screen
    counts, wavelengths and distances: every instance's field and adjoint are
    bitwise those of its own plan with the instance key, and one instance
    matches the oracle."""
    paths = _uneven_sample()
    say("[batch] " + ", ".join(f"N={p.n} M={p.num_screens} R={p.realizations}" for p in paths))
    batch = api.Batch(paths)
    srcs = [c64(np.broadcast_to(workloads.gaussian_source(p.n, p.dx, p.n * p.dx / 8), (p.realizations, p.n, p.n)))
            for p in paths]
    u_in = batch.pack(srcs)
    out, ck = batch.propagate(u_in, seed=7, t=2, checkpoints=True)
    rng = np.random.default_rng(9)
    g = (rng.standard_normal(batch.total) + 1j * rng.standard_normal(batch.total)).astype(np.complex64)
    g_in, g_phi = batch.propagate_backward(c64(g), ck, seed=7, t=2)
    outs, gins = batch.unpack(out), batch.unpack(g_in)
    gs = batch.unpack(c64(g))
    for i, p in enumerate(paths):
        plan = api.Plan(p)
        s_i = api.Batch.instance_seed(7, i)
        o, c = plan.propagate(srcs[i], seed=s_i, t=2, checkpoints=True)
        gi, gp = plan.propagate_backward(gs[i].contiguous(), c, seed=s_i, t=2)
        assert torch.equal(outs[i], o) and torch.equal(gins[i], gi)
        off, size = batch.ck_offsets[i], p.realizations * p.num_screens * p.n * p.n
        assert torch.equal(g_phi[off:off + size].view_as(gp), gp)
        plan.close()
    p = paths[0]
    ref, _ = oracle_propagate(p, api.Batch.instance_seed(7, 0), srcs[0].cpu().numpy(), t=2)
    err = rel_l2(outs[0].cpu().numpy(), ref)
    say(f"[batch] instance 0 vs oracle {err:.2e}")
    assert err < TOL
    batch.close()


def test_graph_replay_reads_device_time(api):
    """One forward step (synthesised screens with subharmonics) captured in a
    HIP graph and replayed with the time step read from device memory: every
    replay, with eager work and synchronisations between replays, equals the
    eager call at that time step bit for bit.  The same for an uneven batch
    (internal streams forked and joined inside the capture)."""
    path = sized_path(256, realizations=4, m=3, sh=3)
    plan, ref = api.Plan(path), api.Plan(path)
    u0 = c64(gaussian(path))
    out = torch.empty((4, path.n, path.n), dtype=torch.complex64, device="cuda")
    t_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.bind_time(t_dev)
    plan.propagate(u0, seed=3, t=0, out=out)  # allocates the workspace before the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.propagate(u0, seed=3, t=0, out=out)
    for t in (4, 1, 9, 1, 0):
        t_dev.fill_(t)
        graph.replay()
        torch.cuda.synchronize()
        got = out.clone()
        want = ref.propagate(u0, seed=3, t=t)
        torch.cuda.synchronize()
        assert torch.equal(got, want), t
    say("[graph] plan: 5 replays equal the eager calls")
    paths = _uneven_sample(4, realizations=(1,))
    batch, eager = api.Batch(paths), api.Batch(paths)
    srcs = [c64(workloads.gaussian_source(p.n, p.dx, p.n * p.dx / 8)[None]) for p in paths]
    ub = batch.pack(srcs)
    ob = torch.empty_like(ub)
    batch.bind_time(t_dev)
    batch.propagate(ub, seed=5, t=0, out=ob)
    torch.cuda.synchronize()
    gb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gb):
        batch.propagate(ub, seed=5, t=0, out=ob)
    for t in (2, 7, 2):
        t_dev.fill_(t)
        gb.replay()
        torch.cuda.synchronize()
        got = ob.clone()
        want = eager.propagate(ub, seed=5, t=t)
        torch.cuda.synchronize()
        assert torch.equal(got, want), t
    say("[graph] batch: 3 replays equal the eager calls")
    plan.bind_time(None)
