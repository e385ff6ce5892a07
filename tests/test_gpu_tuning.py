"""Launch-configuration tuning on the GPU.  Every column-pass and synthesis
width built for a grid size, and every occupancy hint of the screen row
passes, gives bit-identical fields and adjoints (they set the block shape and
the register budget, not the arithmetic), so the parity of the default
choices against the oracle carries over.  The other radix plans round
differently: each is checked against the oracle.  The tuner keeps the fastest
measured configuration, caches it per key and hands it to plans created later."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2604_07248_amd import binding as B
from paper_2604_07248_amd import workloads

from gpu_helpers import TOL, oracle_propagate, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_2604_07248_amd import api as _api
    return _api


@pytest.fixture(autouse=True)
def clean_cache(api):
    api.tune_cache_clear()
    yield
    api.tune_cache_clear()


def c64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def built(n):
    return [k for k in (4, 8, 16) if k <= n and k * n // 16 <= 1024 and (k * n + 2 * n) * 8 <= 160 * 1024]


def sized_path(n, realizations, m, sh=0, **kw):
    lam, dx = 1e-6, (2e-3 if n >= 128 else 4e-3)
    length = min(0.8 * n * dx * dx / lam * m, 2000.0)
    return workloads.uniform_path(n, n * dx, lam, length, m, 1e-15, 0.005, 20.0, sh,
                                  realizations=realizations).with_(**kw)


def evanescent_path():
    return workloads.Path(n=64, dx=0.5e-6, wavelength=1e-6, dz=(4e-6, 7e-6, 4e-6), cn2dz=(2e-17, 2e-17),
                          l0=0.0, L0=float("inf"), tf_kind=workloads.TF_ANGULAR_SPECTRUM, realizations=3)


CASES = {
    "n16": lambda: sized_path(16, 3, 2),
    "n64_sh": lambda: sized_path(64, 3, 2, sh=3),
    "n256": lambda: sized_path(256, 4, 2),
    "n256_angular": lambda: sized_path(256, 3, 2, tf_kind=workloads.TF_ANGULAR_SPECTRUM),
    "n64_evanescent": evanescent_path,
    "n1024": lambda: sized_path(1024, 2, 2, sh=3),
    "n2048": lambda: sized_path(2048, 2, 1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_every_width_bit_identical(api, case):
    path = CASES[case]()
    n, r = path.n, path.realizations
    say(f"[widths] {case} n={n} R={r} widths {built(n)}")
    plan = api.Plan(path)
    u0 = c64(workloads.seeded_field((r, n, n), 21))
    ref, ck = plan.propagate(u0, seed=3, t=1, checkpoints=True)
    g = c64(workloads.seeded_field((r, n, n), 22))
    ref_gin, ref_gphi = plan.propagate_backward(g, ck, seed=3, t=1)
    if case == "n256":
        err = rel_l2(ref.cpu().numpy(), oracle_propagate(path, 3, u0.cpu().numpy(), t=1)[0])
        say(f"[widths] {case} default widths vs oracle {err:.2e}")
        assert err < TOL
    for col in built(n):
        for syn in built(n):
            plan.set_widths(col, syn)
            assert plan.widths == {"col": col, "synth": syn}
            out, ck2 = plan.propagate(u0, seed=3, t=1, checkpoints=True)
            assert torch.equal(out, ref) and torch.equal(ck2, ck), (col, syn)
            if syn == built(n)[0]:
                gin, gphi = plan.propagate_backward(g, ck2, seed=3, t=1)
                assert torch.equal(gin, ref_gin) and torch.equal(gphi, ref_gphi), (col, syn)
    plan.set_widths(0, 0)
    assert plan.widths == {"col": B.plan_widths(plan.handle)[0], "synth": B.plan_widths(plan.handle)[1]}
    plan.close()


RADICES = {512: (8, 4), 1024: (8, 4), 2048: (8,)}


@pytest.mark.parametrize("n", [512, 1024, 2048])
def test_radix_plans_match_oracle(api, n):
    """The second-pass radices built besides the default plan, in the column
    pass and the synthesis: forward and adjoint within 1e-4 of the oracle and
    within rounding of the default plan."""
    r = 2
    path = sized_path(n, r, 2)
    plan = api.Plan(path)
    u0 = c64(workloads.seeded_field((r, n, n), 41))
    g = c64(workloads.seeded_field((r, n, n), 42))
    ref, ck = plan.propagate(u0, seed=6, checkpoints=True)
    ref_gin, _ = plan.propagate_backward(g, ck, seed=6)
    ora = oracle_propagate(path, 6, u0.cpu().numpy())[0]
    for radix in RADICES[n]:
        plan.set_config(col_radix=radix, synth_radix=radix)
        assert plan.config["col_radix"] == radix and plan.config["synth_radix"] == radix
        out, ck2 = plan.propagate(u0, seed=6, checkpoints=True)
        gin, _ = plan.propagate_backward(g, ck2, seed=6)
        e_def = rel_l2(out.cpu().numpy(), ref.cpu().numpy())
        e_ora = rel_l2(out.cpu().numpy(), ora)
        e_g = rel_l2(gin.cpu().numpy(), ref_gin.cpu().numpy())
        say(f"[radix] n={n} R2={radix}: vs default {e_def:.2e}, vs oracle {e_ora:.2e}, adjoint vs default {e_g:.2e}")
        assert e_ora < TOL and e_def < 1e-5 and e_g < 1e-5
    with pytest.raises(B.TurpyError):
        plan.set_config(col_radix=2)
    plan.close()


@pytest.mark.parametrize("n", [256, 1024])
def test_row_occupancy_hints_bit_identical(api, n):
    """The occupancy hints 2, 3, 4 of the forward (relay) and adjoint (pair)
    screen row passes change the register budget only."""
    r = 4
    path = sized_path(n, r, 2, sh=3)
    plan = api.Plan(path)
    u0 = c64(workloads.seeded_field((r, n, n), 51))
    g = c64(workloads.seeded_field((r, n, n), 52))
    ref = plan.propagate(u0, seed=2)
    _, ck = plan.propagate(u0, seed=2, checkpoints=True)
    ref_gin, ref_gphi = plan.propagate_backward(g, ck, seed=2)
    for w in (2, 4):
        plan.set_config(row_waves=w, row_waves_bwd=w)
        assert plan.config["row_waves"] == w and plan.config["row_waves_bwd"] == w
        assert torch.equal(plan.propagate(u0, seed=2), ref)
        gin, gphi = plan.propagate_backward(g, ck, seed=2)
        assert torch.equal(gin, ref_gin) and torch.equal(gphi, ref_gphi)
    plan.set_config()
    assert plan.config["row_waves"] == 3
    with pytest.raises(B.TurpyError):
        api.Plan(sized_path(64, 2, 1)).set_config(row_waves=2)  # hints 2 and 4 are built from N = 256
    plan.close()


def test_tune_measures_caches_and_hands_on(api):
    path = sized_path(512, 8, 2)
    plan = api.Plan(path)
    u0 = c64(workloads.seeded_field((8, 512, 512), 31))
    ref = plan.propagate(u0, seed=4)
    cfg = plan.tune()
    say(f"[tune] n=512 R=8 chose {cfg}; cache {api.tune_cache()}")
    assert cfg == plan.config and cfg["col_width"] in built(512) and cfg["synth_width"] in built(512)
    entries = api.tune_cache()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    keys = {(e["arch"], e["kernel"], e["n"], e["batch_class"]) for e in entries}
    # R = 8: 4 pairs
    assert keys == {(arch, "col_fresnel", 512, 4), (arch, "synth", 512, 3), (arch, "row_fwd", 512, 3),
                    (arch, "row_bwd", 512, 3), (arch, "synth_ar", 512, 3)}
    for e in entries:
        assert 0 < e["us"] <= e["us_default"] * (1 + 1e-6)
        if e["kernel"] in ("col_fresnel", "synth", "synth_ar"):
            assert e["configs"] == len(built(512)) * 3 and e["waves"] == 0
        else:
            assert e["configs"] == 3 and e["width"] == 0 and e["waves"] in (2, 3, 4)
    by = {e["kernel"]: e for e in entries}
    assert (cfg["col_width"], cfg["col_radix"]) == (by["col_fresnel"]["width"], by["col_fresnel"]["radix"])
    assert (cfg["synth_width"], cfg["synth_radix"]) == (by["synth"]["width"], by["synth"]["radix"])
    assert (cfg["ar_width"], cfg["ar_radix"]) == (by["synth_ar"]["width"], by["synth_ar"]["radix"])
    assert (cfg["row_waves"], cfg["row_waves_bwd"]) == (by["row_fwd"]["waves"], by["row_bwd"]["waves"])
    assert rel_l2(plan.propagate(u0, seed=4).cpu().numpy(), ref.cpu().numpy()) < 1e-5
    # a later plan with the same keys starts from the cache; tuning it measures nothing
    plan2 = api.Plan(path)
    assert plan2.config == cfg
    assert plan2.tune() == cfg and api.tune_cache() == entries
    # an entry put by the caller is what the next plan uses
    other = 4 if cfg["col_width"] != 4 else 8
    B.tune_cache_put([{"arch": arch, "kernel": "col_fresnel", "n": 512, "batch_class": 4, "width": other}])
    plan3 = api.Plan(path)
    assert plan3.config["col_width"] == other and plan3.config["col_radix"] == 0 and plan2.config == cfg
    # forced: measured again
    assert plan3.tune(force=True)["col_width"] in built(512)
    assert next(e for e in api.tune_cache() if e["kernel"] == "col_fresnel")["configs"] > 0
    for p in (plan, plan2, plan3):
        p.close()


def test_batch_tune_keeps_results(api):
    paths = [sized_path(n, r, m) for n, r, m in ((256, 2, 2), (1024, 1, 1), (256, 2, 3), (2048, 1, 1))]
    say("[tune] batch " + ", ".join(f"N={p.n} R={p.realizations}" for p in paths))
    batch = api.Batch(paths)
    u_in = batch.pack([c64(workloads.seeded_field((p.realizations, p.n, p.n), 40 + i)) for i, p in enumerate(paths)])
    ref = batch.propagate(u_in, seed=9)
    batch.tune()
    kinds = {(e["kernel"], e["n"]) for e in api.tune_cache()}
    assert {("col_fresnel", n) for n in (256, 1024, 2048)} <= kinds
    assert {("synth", n) for n in (256, 1024, 2048)} <= kinds
    # widths and occupancy hints keep the arithmetic; a tuned radix plan rounds differently
    assert rel_l2(batch.propagate(u_in, seed=9).cpu().numpy(), ref.cpu().numpy()) < 1e-5
    batch.close()


def test_tune_errors(api):
    plan = api.Plan(sized_path(2048, 1, 1))
    for bad in ((16, 0), (0, 16), (5, 0)):
        with pytest.raises(B.TurpyError) as e:
            plan.set_widths(*bad)
        assert e.value.status == B.E_INVALID
    size = B.workspace_size(plan.handle, B.OP_TUNE)
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    st = B.lib().turpy_plan_tune(plan.handle, 0, ctypes.c_void_p(ws.data_ptr()), size - 1, None, None, None)
    assert st == B.E_WORKSPACE
    assert api.tune_cache() == []
    plan.close()
