"""Thin ctypes binding of the device library (include/vtess.h).

Only argument marshalling happens here: every step of the labelling runs in
the HIP kernels of ``libvtess.so``.  PyTorch supplies device memory and the
current stream; no torch type crosses the C ABI.  If the library has not been
built, every entry point raises instead of falling back to anything else.
"""
import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvtess.so")

VORONOI, LAGUERRE, JOHNSON_MEHL = 0, 1, 2
NONPERIODIC, PERIODIC = 0, 1
OK, ERR_INVALID, ERR_NOMEM, ERR_HIP, ERR_BUSY, ERR_INPUT = range(6)
SCALE_MAX, SCALE_MIN = 2.0 ** 200, 2.0 ** -200  # VT_SCALE_MAX / VT_SCALE_MIN
NOALLOC_SCRATCH_BYTES = 64 << 20                # VT_NOALLOC_SCRATCH_BYTES

# Symbols declared in include/vtess.h.
EXPORTS = ["vt_create", "vt_reserve", "vt_destroy", "vt_tessellate", "vt_tessellate_noalloc", "vt_tessellate_nd",
           "vt_tessellate_batch",
           "vt_bins_build",
           "vt_label_batch", "vt_bins_free", "vt_autotune", "vt_load_tuning", "vt_set_params",
           "vt_plan", "vt_plan_nd", "vt_numerics_probe", "vt_label_digest", "vt_profile_enable", "vt_profile_read",
           "vt_status_string", "vt_last_error"]


class VtJob(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("kind", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("L", ctypes.c_double * 3),
                ("growth", ctypes.c_double), ("nsites", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("param", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("keys", ctypes.c_void_p)]


MAX_DIM = 6
ND_GENERIC = 1


class VtJobNd(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("kind", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("n", ctypes.c_int64 * MAX_DIM), ("L", ctypes.c_double * MAX_DIM),
                ("growth", ctypes.c_double), ("nsites", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("param", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("keys", ctypes.c_void_p), ("periods", ctypes.c_void_p)]


class VtError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: status {code} ({status_string(code)}): {last_error()}")
        self.code = code


_lib = None


def lib():
    """Loads libvtess.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"device library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        # PyTorch ships its own HIP runtime under the same soname.  Load it
        # first so that the library binds to that one runtime: tensors and
        # streams then come from the runtime the kernels launch on.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        L.vt_create.argtypes = [ctypes.c_int, P(vp)]
        L.vt_destroy.argtypes = [vp]
        L.vt_destroy.restype = None
        L.vt_tessellate.argtypes = [vp, P(VtJob), vp, vp]
        L.vt_tessellate_noalloc.argtypes = [vp, P(VtJob), vp, vp]
        L.vt_tessellate_nd.argtypes = [vp, P(VtJobNd), vp, vp]
        L.vt_tessellate_batch.argtypes = [vp, P(VtJob), i32, vp, vp]
        L.vt_bins_build.argtypes = [vp, P(VtJob), P(vp), vp, vp]
        L.vt_label_batch.argtypes = [vp, P(vp), i32, vp, vp]
        L.vt_bins_free.argtypes = [vp, vp, vp]
        L.vt_autotune.argtypes = [vp, P(VtJob), i32, ctypes.c_char_p]
        L.vt_load_tuning.argtypes = [vp, ctypes.c_char_p]
        L.vt_set_params.argtypes = [vp, i32, dbl]
        L.vt_plan.argtypes = [vp, P(VtJob), P(i32), P(i32), P(dbl)]
        L.vt_plan_nd.argtypes = [vp, P(VtJobNd), P(i32), P(i32)]
        L.vt_numerics_probe.argtypes = [vp, vp, vp, vp, vp, i64, vp]
        L.vt_label_digest.argtypes = [vp, vp, i64, vp, vp]
        L.vt_reserve.argtypes = [vp, ctypes.c_size_t]
        L.vt_profile_enable.argtypes = [vp, i32]
        L.vt_profile_read.argtypes = [vp, P(dbl), P(dbl), P(dbl), P(i64)]
        L.vt_status_string.argtypes = [ctypes.c_int]
        L.vt_status_string.restype = ctypes.c_char_p
        L.vt_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("vt_destroy", "vt_status_string", "vt_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(code):
    return lib().vt_status_string(int(code)).decode()


def last_error():
    return lib().vt_last_error().decode()


def _check(code, what):
    if code != OK:
        raise VtError(code, what)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_ptr(t, name, dtype, min_numel):
    """Pointer to a contiguous device tensor of `dtype` with at least
    `min_numel` elements (the kernels write that many), else ValueError."""
    import torch
    if t is None:
        return ctypes.c_void_p(0)
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor")
    if t.numel() < min_numel:
        raise ValueError(f"{name} needs at least {min_numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _status_ptr(status, njobs):
    import torch
    return _dev_ptr(status, "status", torch.int32, njobs)


@dataclass
class Job:
    """One diagram: device tensors for sites, parameters and labels."""
    n: tuple
    L: tuple
    kind: int
    periodic: bool
    coords: object            # torch float64 [nsites, ndim] on the device
    param: object = None      # torch float64 [nsites] or None
    growth: float = 1.0
    labels: object = None     # torch int32 with prod(n) elements, allocated if None
    keys: object = None       # torch float64 with prod(n) elements for the distance image, or None
    periods: object = None    # host d x d array-like (row i = period vector L_i) or None

    def _check_tensors(self):
        import torch
        d = len(self.n)
        if self.labels is None:
            self.labels = torch.empty(tuple(reversed(self.n)), dtype=torch.int32,
                                      device=self.coords.device)
        for name, t, dt in (("coords", self.coords, torch.float64), ("param", self.param, torch.float64),
                            ("labels", self.labels, torch.int32), ("keys", self.keys, torch.float64)):
            if t is not None and (t.dtype != dt or not t.is_cuda or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous {dt} device tensor")
        if self.coords.dim() != 2 or self.coords.shape[1] != d:
            raise ValueError("coords must be [nsites, ndim]")
        if self.param is not None and self.param.numel() != self.coords.shape[0]:
            raise ValueError("param must hold one value per site")
        if self.labels.numel() != int(_prod(self.n)):
            raise ValueError("labels must hold prod(n) elements")
        if self.keys is not None and self.keys.numel() != int(_prod(self.n)):
            raise ValueError("keys must hold prod(n) elements")

    def to_c(self):
        d = len(self.n)
        if d not in (2, 3) or self.periods is not None:
            raise ValueError("vt_job holds 2 or 3 axes and orthogonal periods; use Context.tessellate_nd")
        self._check_tensors()
        j = VtJob()
        j.ndim = d
        j.kind = int(self.kind)
        j.bc = PERIODIC if self.periodic else NONPERIODIC
        j.reserved = 0
        for a in range(3):
            j.n[a] = int(self.n[a]) if a < d else 1
            j.L[a] = float(self.L[a]) if a < d else 1.0
        j.growth = float(self.growth)
        j.nsites = int(self.coords.shape[0])
        j.coords = self.coords.data_ptr()
        j.param = self.param.data_ptr() if self.param is not None else None
        j.labels = self.labels.data_ptr()
        j.keys = self.keys.data_ptr() if self.keys is not None else None
        return j

    def to_c_nd(self, generic=False):
        d = len(self.n)
        if not 1 <= d <= MAX_DIM:
            raise ValueError(f"1 to {MAX_DIM} axes")
        self._check_tensors()
        j = VtJobNd()
        j.ndim = d
        j.kind = int(self.kind)
        j.bc = PERIODIC if self.periodic else NONPERIODIC
        j.flags = ND_GENERIC if generic else 0
        for a in range(MAX_DIM):
            j.n[a] = int(self.n[a]) if a < d else 1
            j.L[a] = float(self.L[a]) if a < d else 1.0
        j.growth = float(self.growth)
        j.nsites = int(self.coords.shape[0])
        j.coords = self.coords.data_ptr()
        j.param = self.param.data_ptr() if self.param is not None else None
        j.labels = self.labels.data_ptr()
        j.keys = self.keys.data_ptr() if self.keys is not None else None
        j.periods = None
        if self.periods is not None:
            flat = [float(v) for row in self.periods for v in row]
            if len(flat) != d * d:
                raise ValueError("periods must be ndim x ndim")
            self._periods_buf = (ctypes.c_double * (d * d))(*flat)   # alive while the job is
            j.periods = ctypes.cast(self._periods_buf, ctypes.c_void_p).value
        return j


def plan_scalars(n, L, kind=0, periodic=True, nsites=1, growth=1.0, periods=None, nd=False):
    """Default plan of a job from its scalars alone (vt_plan / vt_plan_nd with
    no context): runs the library's scalar checks and bin planning on the
    host, launches nothing and needs no GPU.  The site, parameter and label
    pointers are placeholders that the planning never reads.  Raises VtError
    (VT_ERR_INVALID) for scalars outside the supported range."""
    d = len(n)
    fake = 256  # never dereferenced
    if not nd and periods is None and d in (2, 3):
        j = VtJob()
        j.ndim, j.kind, j.bc, j.reserved = d, int(kind), PERIODIC if periodic else NONPERIODIC, 0
        for a in range(3):
            j.n[a] = int(n[a]) if a < d else 1
            j.L[a] = float(L[a]) if a < d else 1.0
        j.growth, j.nsites = float(growth), int(nsites)
        j.coords, j.labels = fake, fake
        j.param = fake if kind != VORONOI else None
        nb = (ctypes.c_int32 * 3)()
        cfg = ctypes.c_int32()
        bf = ctypes.c_double()
        _check(lib().vt_plan(None, ctypes.byref(j), nb, ctypes.byref(cfg), ctypes.byref(bf)), "vt_plan")
        return dict(bins=tuple(nb)[:d], tile_cfg=cfg.value, bin_factor=bf.value)
    j = VtJobNd()
    j.ndim, j.kind, j.bc, j.flags = d, int(kind), PERIODIC if periodic else NONPERIODIC, ND_GENERIC
    for a in range(MAX_DIM):
        j.n[a] = int(n[a]) if a < d else 1
        j.L[a] = float(L[a]) if a < d else 1.0
    j.growth, j.nsites = float(growth), int(nsites)
    j.coords, j.labels = fake, fake
    j.param = fake if kind != VORONOI else None
    buf = None
    if periods is not None:
        flat = [float(v) for row in periods for v in row]
        buf = (ctypes.c_double * len(flat))(*flat)
        j.periods = ctypes.cast(buf, ctypes.c_void_p).value
    nb = (ctypes.c_int32 * d)()
    tv = (ctypes.c_int32 * d)()
    _check(lib().vt_plan_nd(None, ctypes.byref(j), nb, tv), "vt_plan_nd")
    return dict(bins=tuple(nb), tile=tuple(tv))


def _prod(v):
    p = 1
    for x in v:
        p *= int(x)
    return p


class Bins:
    """Sites of one job binned on the device; kept until free()."""

    def __init__(self, ctx, handle, job):
        self.ctx, self.handle, self.job = ctx, handle, job

    def free(self, stream=None):
        if self.handle:
            _check(lib().vt_bins_free(self.ctx.handle, self.handle, _stream(stream)), "vt_bins_free")
            self.handle = None


class Context:
    """A vt_ctx on one device."""

    def __init__(self, device=0):
        self.handle = ctypes.c_void_p()
        _check(lib().vt_create(int(device), ctypes.byref(self.handle)), "vt_create")
        self.device = device

    def close(self):
        if self.handle:
            lib().vt_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tessellate(self, job, status=None, stream=None):
        cj = job.to_c()
        _check(lib().vt_tessellate(self.handle, ctypes.byref(cj), _status_ptr(status, 1), _stream(stream)),
               "vt_tessellate")
        return job.labels

    def tessellate_noalloc(self, job, status=None, stream=None):
        """vt_tessellate_noalloc: the plain path on the device's static
        scratch (no device allocation; the labels and status tensors must
        exist already).  Calls on one device must not overlap."""
        if job.labels is None:
            raise ValueError("tessellate_noalloc needs job.labels allocated by the caller")
        cj = job.to_c()
        _check(lib().vt_tessellate_noalloc(self.handle, ctypes.byref(cj), _status_ptr(status, 1),
                                           _stream(stream)), "vt_tessellate_noalloc")
        return job.labels

    def tessellate_nd(self, job, status=None, stream=None, generic=False):
        """Any number of axes from 1 to 6 (vt_tessellate_nd); generic=True
        runs the general kernel also for 2 and 3 axes."""
        cj = job.to_c_nd(generic)
        _check(lib().vt_tessellate_nd(self.handle, ctypes.byref(cj), _status_ptr(status, 1), _stream(stream)),
               "vt_tessellate_nd")
        return job.labels

    def tessellate_batch(self, jobs, status=None, stream=None):
        arr = (VtJob * len(jobs))(*[j.to_c() for j in jobs])
        _check(lib().vt_tessellate_batch(self.handle, arr, len(jobs), _status_ptr(status, len(jobs)),
                                         _stream(stream)),
               "vt_tessellate_batch")
        return [j.labels for j in jobs]

    def bins_build(self, job, status=None, stream=None):
        cj = job.to_c()
        h = ctypes.c_void_p()
        _check(lib().vt_bins_build(self.handle, ctypes.byref(cj), ctypes.byref(h), _status_ptr(status, 1),
                                   _stream(stream)), "vt_bins_build")
        return Bins(self, h, job)

    def label_batch(self, bins, status=None, stream=None):
        arr = (ctypes.c_void_p * len(bins))(*[b.handle for b in bins])
        _check(lib().vt_label_batch(self.handle, arr, len(bins), _status_ptr(status, len(bins)), _stream(stream)),
               "vt_label_batch")

    def autotune(self, samples, cache_path=None):
        arr = (VtJob * len(samples))(*[j.to_c() for j in samples])
        _check(lib().vt_autotune(self.handle, arr, len(samples),
                                 cache_path.encode() if cache_path else None), "vt_autotune")

    def load_tuning(self, path):
        _check(lib().vt_load_tuning(self.handle, path.encode()), "vt_load_tuning")

    def set_params(self, tile_cfg=-1, bin_factor=0.0):
        _check(lib().vt_set_params(self.handle, int(tile_cfg), float(bin_factor)), "vt_set_params")

    def plan(self, job):
        cj = job.to_c()
        nb = (ctypes.c_int32 * 3)()
        cfg = ctypes.c_int32()
        bf = ctypes.c_double()
        _check(lib().vt_plan(self.handle, ctypes.byref(cj), nb, ctypes.byref(cfg), ctypes.byref(bf)),
               "vt_plan")
        return dict(bins=tuple(nb), tile_cfg=cfg.value, bin_factor=bf.value)

    def reserve(self, nbytes):
        """Pre-sizes the context's scratch (synchronises the device once)."""
        _check(lib().vt_reserve(self.handle, int(nbytes)), "vt_reserve")

    def label_digest_async(self, labels, acc, stream=None):
        """Adds the checksum terms of a device int32 label image to `acc` (a
        zeroed int64 device tensor of one element); the checksum is
        int(acc) % (2**31 - 1) once the stream reaches this point."""
        import torch
        lp = _dev_ptr(labels, "labels", torch.int32, 0)
        ap = _dev_ptr(acc, "acc", torch.int64, 1)
        _check(lib().vt_label_digest(self.handle, lp, labels.numel(), ap, _stream(stream)), "vt_label_digest")

    def label_digest(self, labels, stream=None):
        """Checksum of a device label image (waits for the stream)."""
        import torch
        acc = torch.zeros(1, dtype=torch.int64, device=labels.device)
        self.label_digest_async(labels, acc, stream)
        (stream or torch.cuda.current_stream()).synchronize()
        return int(acc.item()) % 2147483647

    def profile_enable(self, enable=True):
        _check(lib().vt_profile_enable(self.handle, 1 if enable else 0), "vt_profile_enable")

    def profile_read(self):
        """(binning ms, main labelling kernel ms, overflow kernel ms, calls)
        summed over the recorded calls."""
        b, l, o, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().vt_profile_read(self.handle, ctypes.byref(b), ctypes.byref(l), ctypes.byref(o),
                                     ctypes.byref(n)), "vt_profile_read")
        return b.value, l.value, o.value, n.value

    def numerics_probe(self, x, den, stream=None):
        """Device sqrt(x) and x / den (binary64), for checking IEEE rounding."""
        import torch
        xp = _dev_ptr(x, "x", torch.float64, 0)
        dp = _dev_ptr(den, "den", torch.float64, x.numel())
        s = torch.empty_like(x)
        q = torch.empty_like(x)
        _check(lib().vt_numerics_probe(self.handle, xp, dp, _ptr(s), _ptr(q), x.numel(),
                                       _stream(stream)), "vt_numerics_probe")
        return s, q
