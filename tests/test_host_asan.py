"""The host-only part of the library (descriptor validation, screen
placement) built with the host compiler's address and undefined-behaviour
sanitizers and driven over valid, malformed and edge-case inputs: no
sanitizer report, and the same statuses, messages and placements as the
hipcc-built library gives for the same inputs."""
import math
import os
import shutil
import subprocess

import pytest

from paper_2604_07248_amd import binding as B
from paper_2604_07248_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_07248_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("asan") / "driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "host.cpp"), os.path.join(CSRC, "planner.cpp"),
           os.path.join(ROOT, "tests", "host_asan_driver.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


def run(driver, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                         timeout=120)
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
    assert res.returncode == 0, res.stderr[-4000:]
    out = res.stdout.splitlines()
    assert len(out) == len(lines)
    return out


def fmt(x):
    return repr(float(x)) if not math.isnan(x) else "nan"


def vline(p, flags=0, no_dz=False, no_cn2=False, m=None):
    m = len(p.cn2dz) if m is None else m
    vals = [flags, p.n, m, p.dx, p.wavelength, p.n0, p.l0, p.L0, p.sh_levels, p.tf_kind, p.inner_scale_conv,
            p.realizations, getattr(p, "psd_alpha", 0.0), int(no_dz), int(no_cn2)]
    arr = list(p.dz) + list(p.cn2dz) if m == len(p.cn2dz) else []
    return "V " + " ".join(fmt(v) for v in vals + arr)


def descriptors():
    base = workloads.config1().path
    limit = base.n * base.dx ** 2 / base.wavelength
    good = [base, workloads.headline(8).path, workloads.config3().path] + \
        [w.path for w in workloads.uneven_batch(instances=12)]
    bad = [base.with_(**c) for c in (
        dict(n=100), dict(n=4096), dict(n=8), dict(dx=0.0), dict(dx=float("nan")), dict(wavelength=-1.0),
        dict(wavelength=float("inf")), dict(n0=0.0), dict(sh_levels=4), dict(sh_levels=-1), dict(tf_kind=7),
        dict(realizations=0), dict(realizations=2 ** 33), dict(inner_scale_conv=3), dict(psd_alpha=1.5),
        dict(psd_alpha=7.0), dict(l0=float("nan")), dict(L0=float("nan")),
        dict(dz=(float("nan"),) + base.dz[1:]), dict(dz=(-1.0,) + base.dz[1:]),
        dict(dz=base.dz[:2] + (0.0,) + base.dz[3:]), dict(dz=base.dz[:-1] + (limit * 1.5,)),
        dict(cn2dz=(-1e-14,) + base.cn2dz[1:]), dict(cn2dz=base.cn2dz[:-1] + (float("inf"),)))]
    lines = [vline(p) for p in good + bad]
    lines += [vline(base, flags=8), vline(base, flags=B.ALLOW_ALIASING | B.CHECK_FINITE | B.SCREEN_CHECKPOINTS),
              vline(base.with_(dz=base.dz[:-1] + (limit * 1.5,)), flags=B.ALLOW_ALIASING),
              vline(base, no_dz=True), vline(base, no_cn2=True), vline(base, m=-1), vline(base, m=(1 << 20) + 1)]
    return lines


def test_validation_under_sanitizers(driver):
    lines = descriptors()
    out = run(driver, lines)
    statuses = [int(o.split()[1]) for o in out]
    assert statuses.count(B.OK) >= 15 and len(set(statuses)) >= 4
    for o in out:
        if int(o.split()[1]) != B.OK:
            assert o.split(" ", 2)[2].startswith("plan_create:"), o


def test_validation_matches_library(driver):
    import ctypes
    base = workloads.config1().path
    limit = base.n * base.dx ** 2 / base.wavelength
    cases = [base.with_(n=100), base.with_(dx=0.0), base.with_(sh_levels=4), base.with_(psd_alpha=7.0),
             base.with_(dz=base.dz[:2] + (0.0,) + base.dz[3:]), base.with_(dz=base.dz[:-1] + (limit * 1.5,)),
             base.with_(cn2dz=(-1e-14,) + base.cn2dz[1:])]
    out = run(driver, [vline(p) for p in cases])
    for p, o in zip(cases, out):
        cp = B.make_cpath(p)
        h = ctypes.c_void_p()
        st = B.lib().turpy_plan_create(ctypes.byref(h), ctypes.byref(cp), 0)
        assert int(o.split()[1]) == st and o.split(" ", 2)[2] == B.last_error(), (o, st, B.last_error())


def placement_cases():
    hv = (B.CN2_HUFNAGEL_VALLEY, 0.0, 1.7e-14, 21.0)
    uni = (B.CN2_UNIFORM, 2e-14, 0.0, 0.0)
    z = [0.0, 400.0, 900.0, 2000.0, 3000.0]
    v = [5e-14, 2e-14, 8e-15, 1e-15, 3e-16]
    cases = []
    for prof, length, lam, n, dx, lim, init in (
            (hv, 3000.0, 1.55e-6, 512, 4e-3, 0.1, 1), (hv, 10000.0, 1.064e-6, 1024, 2e-3, 0.05, 4),
            (uni, 1500.0, 1.064e-6, 1024, 1e-3, 0.1, 2), (uni, 50.0, 5.32e-7, 256, 2e-3, 0.1, 1)):
        cases.append((prof, (), (), length, lam, 1.0, n, dx, lim, init, 256))
    tab = (B.CN2_TABLE, 0.0, 0.0, 0.0)
    cases.append((tab, z, v, 3000.0, 1.55e-6, 1.0, 512, 4e-3, 0.1, 1, 256))
    cases.append((tab, z[:2], v[:2], 3000.0, 1.55e-6, 1.0, 512, 4e-3, 0.1, 1, 256))
    # malformed or too small for the result
    cases.append((hv, (), (), -5.0, 1.55e-6, 1.0, 512, 4e-3, 0.1, 1, 256))
    cases.append((hv, (), (), 3000.0, 1.55e-6, 1.0, 512, 1e-7, 0.1, 1, 256))
    cases.append((hv, (), (), 10000.0, 1.064e-6, 1.0, 1024, 2e-3, 0.05, 4, 1))
    cases.append((tab, [0.0, 10.0, 5.0], [1e-14, 1e-14, 1e-14], 3000.0, 1.55e-6, 1.0, 512, 4e-3, 0.1, 1, 256))
    cases.append((tab, [0.0], [1e-14], 3000.0, 1.55e-6, 1.0, 512, 4e-3, 0.1, 1, 256))
    cases.append(((B.CN2_UNIFORM, -1e-14, 0.0, 0.0), (), (), 1500.0, 1.064e-6, 1.0, 1024, 1e-3, 0.1, 2, 256))
    return cases


def test_placement_under_sanitizers_matches_library(driver):
    cases = placement_cases()
    lines = []
    for prof, z, v, length, lam, n0, n, dx, lim, init, cap in cases:
        vals = list(prof) + [len(z), length, lam, n0, n, dx, lim, init, cap] + list(z) + list(v)
        lines.append("P " + " ".join(fmt(x) for x in vals))
    out = run(driver, lines)
    ok = 0
    for (prof, z, v, length, lam, n0, n, dx, lim, init, cap), o in zip(cases, out):
        f = o.split()
        st = int(f[1])
        zz = (ctypes_array(z), ctypes_array(v))
        cp = B.CCn2Profile(kind=prof[0], cn2=prof[1], A=prof[2], V=prof[3], z=zz[0], values=zz[1], count=len(z))
        try:
            dz, cn2, ry = B.place_screens(cp, length, lam, n0, n, dx, lim, init, capacity=cap)
            lib_st = B.OK
        except B.TurpyError as e:
            lib_st = e.status
        if st == B.E_CAPACITY:
            assert lib_st == B.OK  # the binding retries with the reported count
            continue
        assert st == lib_st, o
        if st == B.OK:
            ok += 1
            m = int(f[2])
            got = [float(x) for x in f[3:]]
            assert m == len(cn2) and len(got) == 3 * m + 1
            for a, b in zip(got, list(dz) + list(cn2) + list(ry)):
                assert a == pytest.approx(b, rel=1e-12, abs=0.0)
    assert ok >= 5


def ctypes_array(vals):
    import ctypes
    if not vals:
        return None
    arr = (ctypes.c_double * len(vals))(*vals)
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)) if arr else None
