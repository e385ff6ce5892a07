"""Thin ctypes binding of libturpy.so (include/turpy.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch supplies device memory (tensors) and the stream.  Loading fails loudly
when the library has not been built; there is no fallback.
"""

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
# TURPY_LIBRARY names another build to load (the tests load the LDS-poison build this way).
LIB_PATH = os.environ.get("TURPY_LIBRARY") or os.path.join(HERE, "libturpy.so")

OK, E_INVALID, E_UNSUPPORTED, E_ALIASING, E_WORKSPACE, E_HIP, E_CAPACITY, E_NONFINITE = range(8)
CN2_UNIFORM, CN2_HUFNAGEL_VALLEY, CN2_TABLE = 0, 1, 2
TF_FRESNEL, TF_ANGULAR_SPECTRUM = 0, 1
SCREENS_SYNTH, SCREENS_MATERIALIZED, SCREENS_SPECTRA = 0, 1, 2
ALLOW_ALIASING = 1
SCREEN_CHECKPOINTS = 2
CHECK_FINITE = 4
OP_SCREEN_GENERATE, OP_PROPAGATE, OP_PROPAGATE_BACKWARD, OP_EVOLVE, OP_PROPAGATE_BACKWARD_REVERSIBLE, OP_TUNE = range(6)
TUNE_COL_FRESNEL, TUNE_COL_ANGULAR, TUNE_COL_AS_TABLE, TUNE_SYNTH, TUNE_ROW_FWD, TUNE_ROW_BWD, TUNE_SYNTH_AR = range(7)
TUNE_KERNELS = ("col_fresnel", "col_angular", "col_as_table", "synth", "row_fwd", "row_bwd", "synth_ar")
TUNE_FORCE = 1

# Every symbol the header declares (checked by the CPU tests).
EXPORTS = [
    "turpy_version", "turpy_last_error", "turpy_plan_create", "turpy_plan_destroy", "turpy_workspace_size",
    "turpy_screen_generate", "turpy_propagate", "turpy_evolve", "turpy_propagate_backward",
    "turpy_propagate_backward_reversible", "turpy_stats",
    "turpy_receiver_workspace_size", "turpy_receiver", "turpy_receiver_backward", "turpy_profile",
    "turpy_profile_only", "turpy_profile_read", "turpy_place_screens", "turpy_state_size", "turpy_plan_bind_time",
    "turpy_batch_create", "turpy_batch_destroy", "turpy_batch_bind_time", "turpy_batch_workspace_size",
    "turpy_batch_propagate", "turpy_batch_propagate_backward", "turpy_plan_tune", "turpy_plan_widths",
    "turpy_plan_set_widths", "turpy_tune_cache_get", "turpy_tune_cache_put", "turpy_tune_cache_clear",
    "turpy_batch_tune", "turpy_plan_config", "turpy_plan_set_config", "turpy_receiver_setup", "turpy_noise", "turpy_propagate_static", "turpy_checkpoint_size", "turpy_evolve_propagate",
    "turpy_plan_bind_moments", "turpy_debug_fail_launch", "turpy_batch_group_limit",
]


class TurpyError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"turpy status {status}: {message}")
        self.status = status


class CPath(ctypes.Structure):
    _fields_ = [
        ("n", c_int32), ("num_screens", c_int32), ("dx", c_double), ("wavelength", c_double), ("n0", c_double),
        ("dz", POINTER(c_double)), ("cn2dz", POINTER(c_double)), ("l0", c_double), ("L0", c_double),
        ("sh_levels", c_int32), ("tf_kind", c_int32), ("inner_scale_conv", c_int32), ("realizations", c_int64),
        ("psd_alpha", c_double),
    ]


class CTuneEntry(ctypes.Structure):
    _fields_ = [
        ("arch", ctypes.c_char * 32), ("kernel", c_int32), ("n", c_int32), ("batch_class", c_int32),
        ("width", c_int32), ("radix", c_int32), ("waves", c_int32), ("configs", c_int32), ("us", c_float),
        ("us_default", c_float),
    ]


class CLaunchConfig(ctypes.Structure):
    _fields_ = [("col_width", c_int32), ("col_radix", c_int32), ("synth_width", c_int32), ("synth_radix", c_int32),
                ("row_waves", c_int32), ("row_waves_bwd", c_int32), ("ar_width", c_int32), ("ar_radix", c_int32)]


class CCn2Profile(ctypes.Structure):
    _fields_ = [
        ("kind", c_int32), ("cn2", c_double), ("A", c_double), ("V", c_double),
        ("z", POINTER(c_double)), ("values", POINTER(c_double)), ("count", c_int64),
    ]


_LIB = None


def _init_torch_gpu():
    """PyTorch ships its own HIP runtime beside the system one the library
    links; the library's runtime finds the device only when PyTorch's has
    initialised first.  Harmless without a GPU or without PyTorch."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """Load libturpy.so once; raises if it is missing or cannot be loaded."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_07248_amd.build`")
        _init_torch_gpu()
        L = ctypes.CDLL(LIB_PATH)
        L.turpy_version.restype = c_char_p
        L.turpy_last_error.restype = c_char_p
        L.turpy_plan_create.argtypes = [POINTER(c_void_p), POINTER(CPath), c_uint32]
        L.turpy_plan_destroy.argtypes = [c_void_p]
        L.turpy_workspace_size.argtypes = [c_void_p, c_int32, POINTER(c_size_t)]
        L.turpy_checkpoint_size.argtypes = [c_void_p, POINTER(c_size_t)]
        L.turpy_evolve_propagate.argtypes = [c_void_p, c_uint64, c_int64, c_double, c_double, c_double, c_void_p,
                                             c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.turpy_screen_generate.argtypes = [c_void_p, c_uint64, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]
        L.turpy_propagate.argtypes = [c_void_p, c_uint64, c_int64, c_void_p, c_int64, c_int32, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_size_t, c_void_p]
        L.turpy_evolve.argtypes = [c_void_p, c_uint64, c_int64, c_double, c_double, c_double, c_void_p, c_void_p,
                                   c_size_t, c_void_p]
        L.turpy_propagate_backward.argtypes = [c_void_p, c_uint64, c_int64, c_void_p, c_void_p, c_int32, c_void_p,
                                               c_void_p, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]
        L.turpy_propagate_backward_reversible.argtypes = [c_void_p, c_uint64, c_int64, c_void_p, c_void_p, c_int32,
                                                          c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_size_t,
                                                          c_void_p]
        L.turpy_stats.argtypes = [c_int32, c_double, c_int64, c_void_p, c_void_p, c_int64, c_int32, c_void_p,
                                  c_double, c_void_p, c_void_p, c_void_p]
        L.turpy_receiver_setup.argtypes = [c_int32]
        L.turpy_propagate_static.argtypes = [c_void_p, c_uint64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                                             c_void_p, c_void_p, c_void_p]
        L.turpy_noise.argtypes = [c_int32, c_int64, c_uint64, c_int64, c_int32, c_int32, c_void_p, c_void_p]
        L.turpy_receiver_workspace_size.argtypes = [c_int32, c_int64, POINTER(c_size_t)]
        L.turpy_receiver.argtypes = [c_int32, c_double, c_double, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_size_t, c_void_p]
        L.turpy_receiver_backward.argtypes = [c_int32, c_double, c_double, c_int64, c_void_p, c_void_p, c_void_p,
                                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.turpy_profile.argtypes = [c_int32]
        L.turpy_profile_only.argtypes = [c_char_p]
        L.turpy_profile_read.argtypes = [c_char_p, POINTER(c_int64), POINTER(c_double)]
        L.turpy_state_size.argtypes = [c_void_p, POINTER(c_size_t)]
        L.turpy_plan_bind_time.argtypes = [c_void_p, c_void_p]
        L.turpy_plan_bind_moments.argtypes = [c_void_p, c_void_p]
        L.turpy_debug_fail_launch.argtypes = [c_int64]
        L.turpy_batch_group_limit.argtypes = [c_size_t]
        L.turpy_batch_create.argtypes = [POINTER(c_void_p), POINTER(CPath), POINTER(c_int64), c_int32, c_uint32]
        L.turpy_batch_destroy.argtypes = [c_void_p]
        L.turpy_batch_bind_time.argtypes = [c_void_p, c_void_p]
        L.turpy_batch_workspace_size.argtypes = [c_void_p, c_int32, POINTER(c_size_t)]
        L.turpy_batch_propagate.argtypes = [c_void_p, c_uint64, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                            c_size_t, c_void_p]
        L.turpy_batch_propagate_backward.argtypes = [c_void_p, c_uint64, c_int64, c_void_p, c_void_p, c_void_p,
                                                     c_void_p, c_void_p, c_size_t, c_void_p]
        L.turpy_place_screens.argtypes = [POINTER(CCn2Profile), c_double, c_double, c_double, c_int32, c_double,
                                          c_double, c_int32, c_int32, POINTER(c_int32), POINTER(c_double),
                                          POINTER(c_double), POINTER(c_double)]
        L.turpy_plan_tune.argtypes = [c_void_p, c_uint32, c_void_p, c_size_t, c_void_p, POINTER(c_int32),
                                      POINTER(c_int32)]
        L.turpy_plan_widths.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32)]
        L.turpy_plan_set_widths.argtypes = [c_void_p, c_int32, c_int32]
        L.turpy_plan_config.argtypes = [c_void_p, POINTER(CLaunchConfig)]
        L.turpy_plan_set_config.argtypes = [c_void_p, POINTER(CLaunchConfig)]
        L.turpy_tune_cache_get.argtypes = [POINTER(CTuneEntry), c_int32, POINTER(c_int32)]
        L.turpy_tune_cache_put.argtypes = [POINTER(CTuneEntry), c_int32]
        L.turpy_tune_cache_clear.argtypes = []
        L.turpy_batch_tune.argtypes = [c_void_p, c_uint32, c_void_p, c_size_t, c_void_p]
        for name in EXPORTS:
            if name not in ("turpy_version", "turpy_last_error"):
                getattr(L, name).restype = c_int32
        _LIB = L
    return _LIB


def check(status):
    if status != OK:
        raise TurpyError(status, lib().turpy_last_error().decode())


def last_error():
    return lib().turpy_last_error().decode()


def make_cpath(path):
    """ctypes descriptor for a workloads.Path (the arrays stay referenced by the result)."""
    m = len(path.cn2dz)
    dz = (c_double * (m + 1))(*path.dz)
    cn2 = (c_double * max(m, 1))(*(path.cn2dz if m else [0.0]))
    cp = CPath(n=path.n, num_screens=m, dx=path.dx, wavelength=path.wavelength, n0=path.n0,
               dz=ctypes.cast(dz, POINTER(c_double)), cn2dz=ctypes.cast(cn2, POINTER(c_double)),
               l0=path.l0, L0=path.L0, sh_levels=path.sh_levels, tf_kind=path.tf_kind,
               inner_scale_conv=path.inner_scale_conv, realizations=path.realizations,
               psd_alpha=getattr(path, "psd_alpha", 0.0))
    cp._keep = (dz, cn2)
    return cp


def plan_create(path, flags=0):
    cp = make_cpath(path)
    handle = c_void_p()
    check(lib().turpy_plan_create(ctypes.byref(handle), ctypes.byref(cp), flags))
    return handle


def batch_create(paths, offsets, flags=0):
    cps = [make_cpath(p) for p in paths]
    arr = (CPath * len(cps))(*cps)
    offs = (c_int64 * len(offsets))(*offsets)
    handle = c_void_p()
    check(lib().turpy_batch_create(ctypes.byref(handle), arr, offs, len(cps), flags))
    return handle


def batch_destroy(handle):
    check(lib().turpy_batch_destroy(handle))


def batch_bind_time(handle, dev_ptr):
    check(lib().turpy_batch_bind_time(handle, dev_ptr))


def batch_workspace_size(handle, op):
    b = c_size_t()
    check(lib().turpy_batch_workspace_size(handle, op, ctypes.byref(b)))
    return b.value


def batch_propagate(handle, seed, t, u_in_ptr, u_out_ptr, ckpt_ptr, ws_ptr, ws_bytes, stream):
    check(lib().turpy_batch_propagate(handle, seed, t, u_in_ptr, u_out_ptr, ckpt_ptr, ws_ptr, ws_bytes, stream))


def batch_propagate_backward(handle, seed, t, gout_ptr, ckpt_ptr, gin_ptr, gscreens_ptr, ws_ptr, ws_bytes, stream):
    check(lib().turpy_batch_propagate_backward(handle, seed, t, gout_ptr, ckpt_ptr, gin_ptr, gscreens_ptr, ws_ptr,
                                               ws_bytes, stream))


def plan_bind_time(handle, dev_ptr):
    check(lib().turpy_plan_bind_time(handle, dev_ptr))


def plan_bind_moments(handle, moments_ptr):
    check(lib().turpy_plan_bind_moments(handle, moments_ptr))


def debug_fail_launch(k):
    check(lib().turpy_debug_fail_launch(k))


def batch_group_limit(nbytes):
    check(lib().turpy_batch_group_limit(nbytes))


def state_size(handle):
    b = c_size_t()
    check(lib().turpy_state_size(handle, ctypes.byref(b)))
    return b.value


def plan_destroy(handle):
    if handle:
        check(lib().turpy_plan_destroy(handle))


def checkpoint_size(handle):
    out = c_size_t()
    check(lib().turpy_checkpoint_size(handle, ctypes.byref(out)))
    return out.value


def workspace_size(handle, op):
    out = c_size_t()
    check(lib().turpy_workspace_size(handle, op, ctypes.byref(out)))
    return out.value


def screen_generate(handle, seed, t, screens_ptr, ws_ptr, ws_bytes, stream):
    check(lib().turpy_screen_generate(handle, seed, t, screens_ptr, ws_ptr, ws_bytes, stream))


def propagate(handle, seed, t, u_in_ptr, u_in_stride, src, screens_ptr, u_out_ptr, ckpt_ptr, ws_ptr, ws_bytes,
              stream):
    check(lib().turpy_propagate(handle, seed, t, u_in_ptr, u_in_stride, src, screens_ptr, u_out_ptr, ckpt_ptr,
                                ws_ptr, ws_bytes, stream))


def evolve(handle, seed, t, alpha, sx, sy, spectra_ptr, ws_ptr, ws_bytes, stream):
    check(lib().turpy_evolve(handle, seed, t, alpha, sx, sy, spectra_ptr, ws_ptr, ws_bytes, stream))


def evolve_propagate(handle, seed, t, alpha, sx, sy, state_ptr, u_in_ptr, u_in_stride, u_out_ptr, ckpt_ptr, ws_ptr,
                     ws_bytes, stream):
    check(lib().turpy_evolve_propagate(handle, seed, t, alpha, sx, sy, state_ptr, u_in_ptr, u_in_stride, u_out_ptr,
                                       ckpt_ptr, ws_ptr, ws_bytes, stream))


def propagate_backward(handle, seed, t, gout_ptr, ckpt_ptr, src, screens_ptr, gin_ptr, gin_stride, gscreens_ptr,
                       ws_ptr, ws_bytes, stream):
    check(lib().turpy_propagate_backward(handle, seed, t, gout_ptr, ckpt_ptr, src, screens_ptr, gin_ptr, gin_stride,
                                         gscreens_ptr, ws_ptr, ws_bytes, stream))


def propagate_backward_reversible(handle, seed, t, gout_ptr, uout_ptr, src, screens_ptr, gin_ptr, gin_stride,
                                  gscreens_ptr, ws_ptr, ws_bytes, stream):
    check(lib().turpy_propagate_backward_reversible(handle, seed, t, gout_ptr, uout_ptr, src, screens_ptr, gin_ptr,
                                                    gin_stride, gscreens_ptr, ws_ptr, ws_bytes, stream))


def stats(n, dx, batch, u_ptr, moments_ptr, count, finalize, si_ptr, summary_ptr, stream, weight_ptr=None,
          power_fraction=0.0):
    check(lib().turpy_stats(n, dx, batch, u_ptr, moments_ptr, count, finalize, weight_ptr, power_fraction, si_ptr,
                            summary_ptr, stream))


def noise(n, pairs, seed, t, tag, screen, out_ptr, stream):
    check(lib().turpy_noise(n, pairs, seed, t, tag, screen, out_ptr, stream))


def receiver_setup(n):
    check(lib().turpy_receiver_setup(n))


def receiver_workspace_size(n, batch):
    out = c_size_t()
    check(lib().turpy_receiver_workspace_size(n, batch, ctypes.byref(out)))
    return out.value


def receiver(n, dx, diameter, batch, u_ptr, th1_ptr, th2_ptr, out_ptr, ws_ptr, ws_bytes, stream):
    check(lib().turpy_receiver(n, dx, diameter, batch, u_ptr, th1_ptr, th2_ptr, out_ptr, ws_ptr, ws_bytes, stream))


def receiver_backward(n, dx, diameter, batch, u_ptr, th1_ptr, th2_ptr, gout_ptr, gu_ptr, g1_ptr, g2_ptr, ws_ptr,
                      ws_bytes, stream):
    check(lib().turpy_receiver_backward(n, dx, diameter, batch, u_ptr, th1_ptr, th2_ptr, gout_ptr, gu_ptr, g1_ptr,
                                        g2_ptr, ws_ptr, ws_bytes, stream))


def profile(enable):
    check(lib().turpy_profile(1 if enable else 0))


def profile_only(family):
    """Time only `family` while profiling (None: every family)."""
    check(lib().turpy_profile_only(family.encode() if family else None))


def profile_read(family):
    n, ms = c_int64(), c_double()
    check(lib().turpy_profile_read(family.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def plan_tune(handle, flags, ws_ptr, ws_bytes, stream):
    col, syn = c_int32(), c_int32()
    check(lib().turpy_plan_tune(handle, flags, ws_ptr, ws_bytes, stream, ctypes.byref(col), ctypes.byref(syn)))
    return col.value, syn.value


def plan_widths(handle):
    col, syn = c_int32(), c_int32()
    check(lib().turpy_plan_widths(handle, ctypes.byref(col), ctypes.byref(syn)))
    return col.value, syn.value


def plan_set_widths(handle, col_width, synth_width):
    check(lib().turpy_plan_set_widths(handle, col_width, synth_width))


CONFIG_FIELDS = ("col_width", "col_radix", "synth_width", "synth_radix", "row_waves", "row_waves_bwd", "ar_width",
                 "ar_radix")


def plan_config(handle):
    c = CLaunchConfig()
    check(lib().turpy_plan_config(handle, ctypes.byref(c)))
    return {f: getattr(c, f) for f in CONFIG_FIELDS}


def plan_set_config(handle, config):
    c = CLaunchConfig(**{f: int(config.get(f, 0)) for f in CONFIG_FIELDS})
    check(lib().turpy_plan_set_config(handle, ctypes.byref(c)))


def batch_tune(handle, flags, ws_ptr, ws_bytes, stream):
    check(lib().turpy_batch_tune(handle, flags, ws_ptr, ws_bytes, stream))


TUNE_FIELDS = ("n", "batch_class", "width", "radix", "waves", "configs")


def tune_cache_get():
    """The tuning cache as a list of dicts (arch, kernel name, n, batch_class,
    width, radix, waves, configs, us, us_default)."""
    count = c_int32()
    check(lib().turpy_tune_cache_get(None, 0, ctypes.byref(count)))
    arr = (CTuneEntry * max(count.value, 1))()
    check(lib().turpy_tune_cache_get(arr, count.value, ctypes.byref(count)))
    out = []
    for e in arr[:count.value]:
        d = {"arch": e.arch.decode(), "kernel": TUNE_KERNELS[e.kernel]}
        d.update({f: getattr(e, f) for f in TUNE_FIELDS})
        d.update({"us": float(e.us), "us_default": float(e.us_default)})
        out.append(d)
    return out


def tune_cache_put(entries):
    """Insert dicts in the form tune_cache_get returns (radix, waves, configs,
    us and us_default optional)."""
    arr = (CTuneEntry * max(len(entries), 1))()
    for i, d in enumerate(entries):
        arch = d["arch"].encode()
        if len(arch) >= 32:
            raise ValueError(f"arch name too long: {d['arch']!r}")
        kernel = d["kernel"]
        arr[i].arch = arch
        arr[i].kernel = TUNE_KERNELS.index(kernel) if isinstance(kernel, str) else int(kernel)
        for f in TUNE_FIELDS:
            setattr(arr[i], f, int(d.get(f, 0)))
        arr[i].us, arr[i].us_default = float(d.get("us", 0.0)), float(d.get("us_default", 0.0))
    check(lib().turpy_tune_cache_put(arr, len(entries)))


def tune_cache_clear():
    check(lib().turpy_tune_cache_clear())


def make_cn2_profile(kind, cn2=0.0, A=0.0, V=0.0, z=None, values=None):
    """ctypes profile descriptor (the table arrays stay referenced by the result)."""
    zt = vt = None
    count = 0
    if z is not None:
        count = len(z)
        zt = (c_double * count)(*z)
        vt = (c_double * count)(*values)
    prof = CCn2Profile(kind=kind, cn2=cn2, A=A, V=V, z=ctypes.cast(zt, POINTER(c_double)) if zt else None,
                       values=ctypes.cast(vt, POINTER(c_double)) if vt else None, count=count)
    prof._keep = (zt, vt)
    return prof


def place_screens(profile, length, wavelength, n0, n, dx, rytov_limit, initial, capacity=256):
    """Returns (dz [M+1], cn2dz [M], rytov [M]) as Python lists; retries once
    with the reported count when `capacity` is too small."""
    m = c_int32()
    for _ in range(2):
        cap = max(int(capacity), 1)
        dz, cn2, ry = (c_double * (cap + 1))(), (c_double * cap)(), (c_double * cap)()
        st = lib().turpy_place_screens(ctypes.byref(profile), length, wavelength, n0, n, dx, rytov_limit, initial,
                                       cap, ctypes.byref(m), dz, cn2, ry)
        if st != E_CAPACITY:
            break
        capacity = m.value
    check(st)
    k = m.value
    return list(dz[:k + 1]), list(cn2[:k]), list(ry[:k])


__all__ = [n for n in dir() if not n.startswith("_")]
_ = (c_float,)
