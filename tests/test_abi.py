"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and rejects invalid descriptors before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2604_07248_amd import binding as B
from paper_2604_07248_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "turpy.h")).read()
    decl = re.findall(r"^\s*(?:turpy_status|const char\*)\s+(turpy_[a-z_]+)\s*\(", text, re.M)
    return sorted(set(decl))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libturpy.so is not built (run __graft_entry__.build())")
    return B.lib()


def test_exports_every_declared_symbol(L):
    declared = header_symbols()
    assert len(declared) >= 13
    assert sorted(B.EXPORTS) == declared
    for name in declared:
        assert getattr(L, name) is not None


def test_version_and_error_strings(L):
    assert b"gfx950" in L.turpy_version()
    assert isinstance(L.turpy_last_error(), bytes)


def _status(path, flags=0):
    cp = B.make_cpath(path)
    h = ctypes.c_void_p()
    st = B.lib().turpy_plan_create(ctypes.byref(h), ctypes.byref(cp), flags)
    return st, B.last_error()


@pytest.mark.parametrize("change,status,needle", [
    (dict(n=100), B.E_INVALID, "power of two"),
    (dict(n=4096), B.E_UNSUPPORTED, "outside"),
    (dict(n=8), B.E_UNSUPPORTED, "outside"),
    (dict(dx=0.0), B.E_INVALID, "dx"),
    (dict(wavelength=-1.0), B.E_INVALID, "wavelength"),
    (dict(sh_levels=4), B.E_UNSUPPORTED, "sh_levels"),
    (dict(tf_kind=7), B.E_INVALID, "tf_kind"),
    (dict(realizations=0), B.E_INVALID, "realizations"),
    (dict(inner_scale_conv=3), B.E_INVALID, "inner_scale_conv"),
    (dict(psd_alpha=1.5), B.E_INVALID, "psd_alpha"),
    (dict(psd_alpha=7.0), B.E_INVALID, "psd_alpha"),
])
def test_invalid_descriptors_rejected(L, change, status, needle):
    p = workloads.config1().path.with_(**change)
    st, msg = _status(p)
    assert st == status and needle in msg, (st, msg)


def test_negative_and_interior_zero_distances(L):
    p = workloads.config1().path
    st, msg = _status(p.with_(dz=(100.0, -1.0, 200.0, 200.0, 200.0, 100.0)))
    assert st == B.E_INVALID and "dz[1]" in msg
    st, msg = _status(p.with_(dz=(100.0, 0.0, 200.0, 200.0, 200.0, 100.0)))
    assert st == B.E_UNSUPPORTED and "merge" in msg
    st, msg = _status(p.with_(cn2dz=(1e-12, -1e-12, 1e-12, 1e-12, 1e-12)))
    assert st == B.E_INVALID and "cn2dz[1]" in msg


def test_aliasing_limit(L):
    """A step beyond N dx^2 n0 / lambda (Sec. 2.4, Eq. 7 at the Nyquist frequency) is refused."""
    p = workloads.config1().path
    limit = p.n * p.dx ** 2 / p.wavelength
    st, msg = _status(p.with_(dz=(100.0, 200.0, 200.0, 200.0, limit * 1.01, 100.0)))
    assert st == B.E_ALIASING and "sampling limit" in msg


def test_stats_argument_errors(L):
    st = L.turpy_stats(64, 0.01, 1, None, None, 0, 0, None, 0.0, None, None, None)
    assert st == B.E_INVALID and "moments" in B.last_error()
    st = L.turpy_stats(0, 0.01, 0, None, None, 0, 0, None, 0.0, None, None, None)
    assert st == B.E_INVALID
    # a non-NULL moments pointer is only checked for NULL before validation ends
    fake = ctypes.c_void_p(256)
    st = L.turpy_stats(64, 0.01, 0, None, fake, 1, 1, None, 1.5, None, fake, None)
    assert st == B.E_INVALID and "power_fraction" in B.last_error()


def test_receiver_needs_setup(L):
    """Plan-less receiver calls allocate nothing: their tables come from
    turpy_receiver_setup, and a call for an n never set up is refused before
    anything is enqueued."""
    fake = ctypes.c_void_p(256)
    other = ctypes.c_void_p(512)
    st = L.turpy_receiver(32, 0.01, 0.3, 1, fake, fake, fake, other, None, 0, None)
    assert st in (B.E_INVALID, B.E_HIP)
    if st == B.E_INVALID:
        assert "turpy_receiver_setup" in B.last_error()


def test_status_and_flag_values_match_header(L):
    text = open(os.path.join(ROOT, "include", "turpy.h")).read()
    status = dict((k, int(v)) for k, v in re.findall(r"TURPY_(E_[A-Z]+|OK) = (\d+)", text))
    for name, value in status.items():
        assert getattr(B, name) == value, name
    flags = dict((k, int(v)) for k, v in re.findall(r"#define TURPY_([A-Z_]+) (\d+)u", text))
    for name in ("ALLOW_ALIASING", "SCREEN_CHECKPOINTS", "CHECK_FINITE"):
        assert getattr(B, name) == flags[name], name
    assert len(set(flags[n] for n in ("ALLOW_ALIASING", "SCREEN_CHECKPOINTS", "CHECK_FINITE"))) == 3


def test_unknown_plan_flags_rejected(L):
    st, msg = _status(workloads.config1().path, flags=8)
    assert st == B.E_INVALID and "flags" in msg


def test_debug_fail_launch_arguments(L):
    assert L.turpy_debug_fail_launch(-1) == B.E_INVALID
    assert L.turpy_debug_fail_launch(0) == B.OK
    assert L.turpy_plan_bind_moments(None, None) == B.E_INVALID


def test_empty_batch_rejected(L):
    h = ctypes.c_void_p()
    st = L.turpy_batch_create(ctypes.byref(h), None, None, 0, 0)
    assert st == B.E_INVALID and "num_paths" in B.last_error()
    assert not h.value
