"""PyTorch-facing wrapper of the HIP library: plans, tensors and streams.

Everything numeric happens inside libturpy.so; this module only checks
shapes, allocates output tensors and passes device pointers and the current
HIP stream.
"""

import ctypes
import json
import os

import torch

from . import binding as B


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# Library handles released while the current stream is being captured into a
# graph (for instance by the garbage collector, inside a torch.cuda.graph
# block) are destroyed after the capture: destroying one frees device memory,
# which would invalidate the capture.
_deferred = []


def _capturing():
    try:
        return torch.cuda.is_current_stream_capturing()
    except Exception:
        return False


def _flush_deferred():
    if not _deferred or _capturing():
        return
    pending = list(_deferred)
    del _deferred[:]
    for destroy, handle in pending:
        destroy(handle)


def _release(destroy, handle):
    if _capturing():
        _deferred.append((destroy, handle))
    else:
        _flush_deferred()
        destroy(handle)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on the GPU, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")


class Plan:
    """A propagation plan for one path (workloads.Path) on the current device."""

    def __init__(self, path, flags=0, device=None):
        self.path = path
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        tune_cache_from_env()
        _flush_deferred()
        with torch.cuda.device(self.device):
            self.handle = B.plan_create(path, flags)
        self.flags = flags
        self.n, self.m, self.r = path.n, len(path.cn2dz), path.realizations
        self.pairs = (self.r + 1) // 2
        self._ws = {}

    # -- checkpoints -----------------------------------------------------------
    @property
    def keeps_screens(self):
        """Plan created with binding.SCREEN_CHECKPOINTS: the checkpoints also
        hold the screens' column halves (the adjoint does not synthesise them)."""
        return bool(self.flags & B.SCREEN_CHECKPOINTS)

    def new_checkpoints(self):
        """An empty checkpoint buffer: complex64 [R][M][N][N], or, when the plan
        keeps the screens, a flat complex64 buffer of turpy_checkpoint_size bytes
        (checkpoint_fields gives its [R][M][N][N] part)."""
        if self.keeps_screens:
            return torch.empty(B.checkpoint_size(self.handle) // 8, dtype=torch.complex64, device=self.device)
        return torch.empty((self.r, self.m, self.n, self.n), dtype=torch.complex64, device=self.device)

    def checkpoint_fields(self, ck):
        """The fields after each screen, [R][M][N][N], of a checkpoint buffer."""
        return ck.reshape(-1)[: self.r * self.m * self.n * self.n].view(self.r, self.m, self.n, self.n)

    def _need_ck(self, ck):
        if self.keeps_screens:
            _need(ck, torch.complex64, (B.checkpoint_size(self.handle) // 8,), "checkpoints")
        else:
            _need(ck, torch.complex64, (self.r, self.m, self.n, self.n), "checkpoints")

    def close(self):
        handle = getattr(self, "handle", None)
        if handle:
            self.handle = None
            _release(B.plan_destroy, handle)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bind_time(self, t_dev):
        """Read the noise time step from a one-element int32/uint32 CUDA tensor
        when the kernels run (graph replays); None restores the argument."""
        if t_dev is not None:
            if t_dev.numel() != 1 or t_dev.element_size() != 4 or not t_dev.is_cuda:
                raise ValueError("bind_time: a one-element 4-byte integer tensor on the GPU")
        self._t_dev = t_dev  # kept alive while bound
        B.plan_bind_time(self.handle, _ptr(t_dev))

    def bind_moments(self, moments):
        """Take the ensemble moments inside every forward call (a Moments of
        this plan's N on its device, or None to stop): each call adds its R
        output fields, with the bits of moments.add(u_out), and counts them."""
        if moments is not None:
            if not isinstance(moments, Moments) or moments.n != self.n or moments.device != self.device:
                raise ValueError("bind_moments: a Moments of the plan's grid size on its device")
        self._moments = moments  # kept alive while bound
        B.plan_bind_moments(self.handle, _ptr(moments.buf) if moments is not None else None)

    def _counted(self):
        if getattr(self, "_moments", None) is not None:
            self._moments.count += self.r

    def workspace(self, op):
        size = B.workspace_size(self.handle, op)
        buf = self._ws.get(op)
        if buf is None or buf.numel() < size:
            buf = torch.empty(max(size, 256), dtype=torch.uint8, device=self.device)
            self._ws[op] = buf
        return buf, size

    # -- launch shapes -------------------------------------------------------
    def tune(self, force=False):
        """Time the launch configurations of the column pass, the synthesis
        (plain and with the AR step fused) and the screen row passes
        (turpy_plan_tune; synchronises) and keep the
        fastest, or take them from the tuning cache.  Returns the plan's
        launch configuration (config)."""
        size = B.workspace_size(self.handle, B.OP_TUNE)
        ws = torch.empty(max(size, 256), dtype=torch.uint8, device=self.device)
        B.plan_tune(self.handle, B.TUNE_FORCE if force else 0, _ptr(ws), size, _stream())
        del ws
        _tune_cache_to_env()
        return self.config

    @property
    def config(self):
        """Every launch choice: col_width, col_radix, synth_width, synth_radix,
        row_waves, row_waves_bwd, ar_width, ar_radix (the synthesis with the AR
        step fused)."""
        return B.plan_config(self.handle)

    def set_config(self, **choices):
        """Set launch choices (missing or 0: the built-in choice)."""
        B.plan_set_config(self.handle, choices)

    @property
    def widths(self):
        """The strip widths the plan's launches use: {"col": K, "synth": K}."""
        col, syn = B.plan_widths(self.handle)
        return {"col": col, "synth": syn}

    def set_widths(self, col=0, synth=0):
        """Set the strip widths (0: the built-in choice for N)."""
        B.plan_set_widths(self.handle, col, synth)

    # -- screens -------------------------------------------------------------
    def screens(self, seed, t=0, out=None):
        """Phase screens float32 [R][M][N][N] (radians)."""
        shape = (self.r, self.m, self.n, self.n)
        out = torch.empty(shape, dtype=torch.float32, device=self.device) if out is None else out
        _need(out, torch.float32, shape, "screens")
        ws, size = self.workspace(B.OP_SCREEN_GENERATE)
        B.screen_generate(self.handle, seed, t, _ptr(out), _ptr(ws), size, _stream())
        return out

    def init_spectra(self, seed):
        """AR state at t = 0: the pair spectra complex64 [ceil(R/2)][M][N][N]
        (radians), a view at the start of a buffer that also holds the
        subharmonic coefficients when the plan has subharmonic levels
        (`sh_coefficients`)."""
        elems = B.state_size(self.handle) // 8
        buf = torch.empty(elems, dtype=torch.complex64, device=self.device)
        spec = buf[: self.pairs * self.m * self.n * self.n].view(self.pairs, self.m, self.n, self.n)
        B.evolve(self.handle, seed, 0, 0.0, 0.0, 0.0, _ptr(spec), None, 0, _stream())
        return spec

    def _need_state(self, spectra):
        _need(spectra, torch.complex64, (self.pairs, self.m, self.n, self.n), "spectra")
        room = spectra.untyped_storage().nbytes() - spectra.storage_offset() * spectra.element_size()
        if room < B.state_size(self.handle):
            raise ValueError("spectra: the AR state needs room for the subharmonic coefficients after the "
                             "spectra; allocate it with init_spectra")

    def sh_coefficients(self, spectra):
        """The state's subharmonic block complex64 [ceil(R/2)][M][32] (radians;
        24 coefficients, their grid mean, padding), or None without levels."""
        self._need_state(spectra)
        if self.path.sh_levels == 0 or self.m == 0:
            return None
        base = spectra.storage_offset() + spectra.numel()
        return torch.empty(0, dtype=torch.complex64, device=self.device).set_(
            spectra.untyped_storage(), base, (self.pairs, self.m, 32))

    def evolve(self, spectra, seed, t, alpha, shift_x=0.0, shift_y=0.0):
        self._need_state(spectra)
        if t < 1:
            raise ValueError("evolve: t must be >= 1 (t = 0 is init_spectra)")
        B.evolve(self.handle, seed, t, alpha, shift_x, shift_y, _ptr(spectra), None, 0, _stream())
        return spectra

    # -- propagation -----------------------------------------------------------
    def _source(self, u_in):
        if u_in.dim() == 2:
            _need(u_in, torch.complex64, (self.n, self.n), "u_in")
            return 0
        _need(u_in, torch.complex64, (self.r, self.n, self.n), "u_in")
        return self.n * self.n

    def _screen_src(self, screens, spectra):
        if screens is not None and spectra is not None:
            raise ValueError("give screens or spectra, not both")
        if screens is not None:
            _need(screens, torch.float32, (self.r, self.m, self.n, self.n), "screens")
            return B.SCREENS_MATERIALIZED, screens
        if spectra is not None:
            self._need_state(spectra)
            return B.SCREENS_SPECTRA, spectra
        return B.SCREENS_SYNTH, None

    def propagate(self, u_in, seed=0, t=0, screens=None, spectra=None, checkpoints=False, out=None):
        """Forward split-step; returns u_out [R][N][N], and the checkpoints [R][M][N][N]
        when `checkpoints` is True (allocated) or a tensor (filled)."""
        stride = self._source(u_in)
        src, sbuf = self._screen_src(screens, spectra)
        shape = (self.r, self.n, self.n)
        u_out = torch.empty(shape, dtype=torch.complex64, device=self.device) if out is None else out
        _need(u_out, torch.complex64, shape, "u_out")
        ck = None
        if isinstance(checkpoints, torch.Tensor):
            ck = checkpoints
            self._need_ck(ck)
        elif checkpoints:
            ck = self.new_checkpoints()
        ws, size = self.workspace(B.OP_PROPAGATE)
        B.propagate(self.handle, seed, t, _ptr(u_in), stride, src, _ptr(sbuf), _ptr(u_out), _ptr(ck), _ptr(ws), size,
                    _stream())
        self._counted()
        return (u_out, ck) if ck is not None else u_out

    def evolve_propagate(self, spectra, seed, t, alpha, shift_x=0.0, shift_y=0.0, u_in=None, checkpoints=False,
                         out=None):
        """One AR time step: evolve(spectra, seed, t, ...) then
        propagate(u_in, spectra=spectra), with the evolution fused into the
        screen synthesis (turpy_evolve_propagate).  Returns like propagate."""
        self._need_state(spectra)
        if t < 1:
            raise ValueError("evolve_propagate: t must be >= 1 (t = 0 is init_spectra)")
        stride = self._source(u_in)
        shape = (self.r, self.n, self.n)
        u_out = torch.empty(shape, dtype=torch.complex64, device=self.device) if out is None else out
        _need(u_out, torch.complex64, shape, "u_out")
        ck = None
        if isinstance(checkpoints, torch.Tensor):
            ck = checkpoints
            self._need_ck(ck)
        elif checkpoints:
            ck = self.new_checkpoints()
        ws, size = self.workspace(B.OP_PROPAGATE)
        B.evolve_propagate(self.handle, seed, t, alpha, shift_x, shift_y, _ptr(spectra), _ptr(u_in), stride,
                           _ptr(u_out), _ptr(ck), _ptr(ws), size, _stream())
        self._counted()
        return (u_out, ck) if ck is not None else u_out

    def propagate_backward(self, grad_out, checkpoints, seed=0, t=0, screens=None, spectra=None, want_input=True,
                           want_screens=True, u_out=None, shared_source=False):
        """Adjoint of propagate.  With checkpoints=None and the forward output
        u_out, the screen-plane fields are rebuilt from u_out instead
        (turpy_propagate_backward_reversible).  shared_source=True returns the
        gradient of a source shared by every realization, [N][N] (the library
        sums over realizations)."""
        shape = (self.r, self.n, self.n)
        _need(grad_out, torch.complex64, shape, "grad_out")
        src, sbuf = self._screen_src(screens, spectra)
        reversible = checkpoints is None and u_out is not None
        if reversible:
            _need(u_out, torch.complex64, shape, "u_out")
        elif self.m > 0:
            self._need_ck(checkpoints)
        g_shape = (self.n, self.n) if shared_source else shape
        g_stride = 0 if shared_source else self.n * self.n
        g_in = torch.empty(g_shape, dtype=torch.complex64, device=self.device) if want_input else None
        g_phi = (torch.empty((self.r, self.m, self.n, self.n), dtype=torch.float32, device=self.device)
                 if want_screens else None)
        if reversible:
            ws, size = self.workspace(B.OP_PROPAGATE_BACKWARD_REVERSIBLE)
            B.propagate_backward_reversible(self.handle, seed, t, _ptr(grad_out), _ptr(u_out), src, _ptr(sbuf),
                                            _ptr(g_in), g_stride, _ptr(g_phi), _ptr(ws), size, _stream())
        else:
            ws, size = self.workspace(B.OP_PROPAGATE_BACKWARD)
            B.propagate_backward(self.handle, seed, t, _ptr(grad_out), _ptr(checkpoints), src, _ptr(sbuf),
                                 _ptr(g_in), g_stride, _ptr(g_phi), _ptr(ws), size, _stream())
        return g_in, g_phi


SEED_STEP = 0x9E3779B97F4A7C15


class Batch:
    """An uneven batch of path instances (turpy_batch_*): every instance has
    its own grid size, screen count and distances; their fields live in one
    packed complex64 buffer (instance i at offsets[i], [R_i][N_i][N_i]).
    Instance i draws the noise of a single plan keyed (seed + i * SEED_STEP)
    mod 2^64."""

    def __init__(self, paths, flags=0, device=None):
        self.paths = list(paths)
        sizes = [p.realizations * p.n * p.n for p in self.paths]
        self.offsets = [0]
        for sz in sizes[:-1]:
            self.offsets.append(self.offsets[-1] + sz)
        self.total = sum(sizes)
        ck = [p.realizations * len(p.cn2dz) * p.n * p.n for p in self.paths]
        self.ck_offsets = [0]
        for c in ck[:-1]:
            self.ck_offsets.append(self.ck_offsets[-1] + c)
        self.ck_total = sum(ck)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        tune_cache_from_env()
        _flush_deferred()
        with torch.cuda.device(self.device):
            self.handle = B.batch_create(self.paths, self.offsets, flags)
        self._ws = {}

    def close(self):
        handle = getattr(self, "handle", None)
        if handle:
            self.handle = None
            _release(B.batch_destroy, handle)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def instance_seed(seed, i):
        return (seed + i * SEED_STEP) % (1 << 64)

    def pack(self, fields):
        """Packed buffer from per-instance complex64 tensors [R_i][N_i][N_i]."""
        return torch.cat([f.reshape(-1) for f in fields]).to(self.device)

    def unpack(self, flat):
        """Per-instance views [R_i][N_i][N_i] of a packed buffer."""
        return [flat[o:o + p.realizations * p.n * p.n].view(p.realizations, p.n, p.n)
                for o, p in zip(self.offsets, self.paths)]

    def bind_time(self, t_dev):
        """As Plan.bind_time, for every instance."""
        if t_dev is not None and (t_dev.numel() != 1 or t_dev.element_size() != 4 or not t_dev.is_cuda):
            raise ValueError("bind_time: a one-element 4-byte integer tensor on the GPU")
        self._t_dev = t_dev
        B.batch_bind_time(self.handle, _ptr(t_dev))

    def _workspace(self, op):
        size = B.batch_workspace_size(self.handle, op)
        buf = self._ws.get(op)
        if buf is None or buf.numel() < size:
            buf = torch.empty(max(size, 256), dtype=torch.uint8, device=self.device)
            self._ws[op] = buf
        return buf, size

    def tune(self, force=False):
        """Plan.tune for every instance; each distinct key is measured once."""
        size = B.batch_workspace_size(self.handle, B.OP_TUNE)
        ws = torch.empty(max(size, 256), dtype=torch.uint8, device=self.device)
        B.batch_tune(self.handle, B.TUNE_FORCE if force else 0, _ptr(ws), size, _stream())
        del ws
        _tune_cache_to_env()

    def propagate(self, u_in, seed=0, t=0, checkpoints=False, out=None):
        _need(u_in, torch.complex64, (self.total,), "u_in")
        out = torch.empty_like(u_in) if out is None else out
        _need(out, torch.complex64, (self.total,), "out")
        ck = None
        if isinstance(checkpoints, torch.Tensor):
            ck = checkpoints
            _need(ck, torch.complex64, (self.ck_total,), "checkpoints")
        elif checkpoints:
            ck = torch.empty(self.ck_total, dtype=torch.complex64, device=self.device)
        ws, size = self._workspace(B.OP_PROPAGATE)
        B.batch_propagate(self.handle, seed, t, _ptr(u_in), _ptr(out), _ptr(ck), _ptr(ws), size, _stream())
        return (out, ck) if ck is not None else out

    def propagate_backward(self, grad_out, checkpoints, seed=0, t=0, grad_in=None, grad_screens=None):
        """Adjoint of propagate: (dL/du_in packed like the fields, dL/dphi
        packed like the checkpoints); the output tensors may be given."""
        _need(grad_out, torch.complex64, (self.total,), "grad_out")
        _need(checkpoints, torch.complex64, (self.ck_total,), "checkpoints")
        g_in = torch.empty_like(grad_out) if grad_in is None else grad_in
        _need(g_in, torch.complex64, (self.total,), "grad_in")
        g_phi = (torch.empty(self.ck_total, dtype=torch.float32, device=self.device) if grad_screens is None
                 else grad_screens)
        _need(g_phi, torch.float32, (self.ck_total,), "grad_screens")
        ws, size = self._workspace(B.OP_PROPAGATE_BACKWARD)
        B.batch_propagate_backward(self.handle, seed, t, _ptr(grad_out), _ptr(checkpoints), _ptr(g_in), _ptr(g_phi),
                                   _ptr(ws), size, _stream())
        return g_in, g_phi


def noise(n, pairs, seed, t=0, tag=1, screen=0, out=None, device=None):
    """The complex normals N_c of a spectrum, complex64 [pairs][n][n]
    (turpy_noise: the numbers the synthesis draws for (seed, t, tag, screen))."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((pairs, n, n), dtype=torch.complex64, device=dev) if out is None else out
    _need(out, torch.complex64, (pairs, n, n), "out")
    B.noise(n, pairs, seed, t, tag, screen, _ptr(out), _stream())
    return out


TUNE_CACHE_FORMAT = "turpy-tune-cache"
TUNE_CACHE_VERSION = 2


def tune_cache():
    """Entries of the process-wide tuning cache (list of dicts)."""
    return B.tune_cache_get()


def tune_cache_save(path):
    """Write the tuning cache as JSON."""
    with open(path, "w") as f:
        json.dump({"format": TUNE_CACHE_FORMAT, "version": TUNE_CACHE_VERSION, "entries": B.tune_cache_get()}, f,
                  indent=1)


def tune_cache_load(path):
    """Merge a JSON file written by tune_cache_save into the cache; returns
    the number of entries read.  Plans created afterwards use them."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != TUNE_CACHE_FORMAT or doc.get("version") != TUNE_CACHE_VERSION:
        raise ValueError(f"{path}: not a version-{TUNE_CACHE_VERSION} {TUNE_CACHE_FORMAT} file")
    B.tune_cache_put(doc["entries"])
    return len(doc["entries"])


def tune_cache_clear():
    B.tune_cache_clear()


TUNE_CACHE_ENV = "TURPY_TUNE_CACHE"
_env_cache_read = []


def tune_cache_from_env():
    """Merge the JSON file named by $TURPY_TUNE_CACHE into the cache, once per
    process (plans and batches call this before they are created; a missing
    file is skipped).  Returns the number of entries read."""
    path = os.environ.get(TUNE_CACHE_ENV)
    if not path or path in _env_cache_read:
        return 0
    _env_cache_read.append(path)
    return tune_cache_load(path) if os.path.exists(path) else 0


def _tune_cache_to_env():
    path = os.environ.get(TUNE_CACHE_ENV)
    if path:
        tune_cache_save(path)


class Moments:
    """Running ensemble moments of |U|^2 on the GPU (turpy_stats)."""

    def __init__(self, n, dx, device=None):
        self.n, self.dx = n, dx
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.buf = torch.zeros((4, n, n), dtype=torch.float32, device=self.device)
        self.count = 0

    def add(self, u):
        if u.dim() == 2:
            u = u.unsqueeze(0)
        _need(u, torch.complex64, (u.shape[0], self.n, self.n), "u")
        B.stats(self.n, self.dx, u.shape[0], _ptr(u), _ptr(self.buf), 0, 0, None, None, _stream())
        self.count += u.shape[0]

    def finalize(self, weight=None, power_fraction=0.0):
        """SI map and summary.  The SI entries are taken over the central
        region, or with power_fraction > 0 over the power-cutoff region of
        Sec. 4.1 (0.999 there); weight: optional float32 [N][N] weights."""
        if weight is not None:
            _need(weight, torch.float32, (self.n, self.n), "weight")
        si = torch.empty((self.n, self.n), dtype=torch.float32, device=self.device)
        summary = torch.empty(8, dtype=torch.float64, device=self.device)
        B.stats(self.n, self.dx, 0, None, _ptr(self.buf), self.count, 1, _ptr(si), _ptr(summary), _stream(),
                _ptr(weight), power_fraction)
        s = summary.cpu().tolist()
        return si, {"si_plane": s[0], "w_2nd": s[1], "w_fit": s[2], "count": int(s[3]), "si_sum": s[4],
                    "region_weight": s[5], "threshold": s[6]}


class Receiver:
    """Dual-domain two-mask receiver on an N x N grid (turpy_receiver)."""

    def __init__(self, n, dx, aperture_diameter=0.3048, device=None):
        self.n, self.dx, self.diameter = n, dx, aperture_diameter
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self._ws = None
        with torch.cuda.device(self.device):
            B.receiver_setup(n)

    def forward(self, u, theta1, theta2, out=None):
        b = u.shape[0]
        _need(u, torch.complex64, (b, self.n, self.n), "u")
        _need(theta1, torch.float32, (self.n, self.n), "theta1")
        _need(theta2, torch.float32, (self.n, self.n), "theta2")
        out = torch.empty_like(u) if out is None else out
        B.receiver(self.n, self.dx, self.diameter, b, _ptr(u), _ptr(theta1), _ptr(theta2), _ptr(out), None, 0,
                   _stream())
        return out

    def backward(self, u, theta1, theta2, grad_out, want_u=True):
        b = u.shape[0]
        _need(grad_out, torch.complex64, (b, self.n, self.n), "grad_out")
        size = B.receiver_workspace_size(self.n, b)
        if self._ws is None or self._ws.numel() < size:
            self._ws = torch.empty(size, dtype=torch.uint8, device=self.device)
        g_u = torch.empty_like(u) if want_u else None
        g1 = torch.empty((self.n, self.n), dtype=torch.float32, device=self.device)
        g2 = torch.empty((self.n, self.n), dtype=torch.float32, device=self.device)
        B.receiver_backward(self.n, self.dx, self.diameter, b, _ptr(u), _ptr(theta1), _ptr(theta2), _ptr(grad_out),
                            _ptr(g_u), _ptr(g1), _ptr(g2), _ptr(self._ws), size, _stream())
        return g_u, g1, g2


class ReceiverFn(torch.autograd.Function):
    """u_out = receiver(u, theta1, theta2) with the hand-written adjoint."""

    @staticmethod
    def forward(ctx, u, theta1, theta2, rx):
        u, theta1, theta2 = u.contiguous(), theta1.contiguous(), theta2.contiguous()
        ctx.rx = rx
        ctx.save_for_backward(u, theta1, theta2)
        return rx.forward(u, theta1, theta2)

    @staticmethod
    def backward(ctx, grad_out):
        u, theta1, theta2 = ctx.saved_tensors
        g_u, g1, g2 = ctx.rx.backward(u, theta1, theta2, grad_out.contiguous(), want_u=ctx.needs_input_grad[0])
        return g_u, g1, g2, None


class Propagate(torch.autograd.Function):
    """u_out = propagate(u_in, phi) with the hand-written adjoint as backward.

    Fields are checkpointed at the screen planes only (or, with
    reversible=True, rebuilt from the output in the backward: no checkpoint
    memory); the backward regenerates synthesised screens from (seed, t).
    `screens` may be None (synthesised) or a float32 [R][M][N][N] tensor
    (materialised; receives dL/dphi)."""

    @staticmethod
    def forward(ctx, u_in, screens, plan, seed, t, reversible=False):
        scr = screens.contiguous() if screens is not None else None
        if reversible:
            u_out = plan.propagate(u_in.contiguous(), seed, t, screens=scr)
            ctx.save_for_backward(u_out, screens)
        else:
            u_out, ck = plan.propagate(u_in.contiguous(), seed, t, screens=scr, checkpoints=True)
            ctx.save_for_backward(ck, screens)
        ctx.plan, ctx.seed, ctx.t, ctx.reversible = plan, seed, t, reversible
        ctx.shared = u_in.dim() == 2
        return u_out

    @staticmethod
    def backward(ctx, grad_out):
        saved, screens = ctx.saved_tensors
        plan = ctx.plan
        want_in = ctx.needs_input_grad[0]
        want_phi = ctx.needs_input_grad[1] or screens is None
        kw = {"u_out": saved} if ctx.reversible else {}
        g_in, g_phi = plan.propagate_backward(grad_out.contiguous(), None if ctx.reversible else saved, ctx.seed,
                                              ctx.t, screens=screens, want_input=want_in,
                                              want_screens=want_phi and screens is not None,
                                              shared_source=ctx.shared, **kw)
        return g_in, (g_phi if screens is not None and ctx.needs_input_grad[1] else None), None, None, None, None
