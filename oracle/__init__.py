"""CPU oracle for digital Voronoi, Laguerre and Johnson-Mehl diagrams.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the device library and
its Python binding never do.  The oracle is plain C (``vto.c``) following the
paper's algorithms (arXiv 2201.13234, Sec. 3) in IEEE binary64; this module
only marshals numpy arrays into it.
"""
import ctypes
import math
import os

import numpy as np

from .build import LIB

VORONOI, LAGUERRE, JOHNSON_MEHL = 0, 1, 2
OK, ERR_INVALID, ERR_NOMEM, ERR_INPUT = 0, 1, 2, 5
MAX_DIM = 6


class Problem(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("lattice", ctypes.c_int32),
                ("n", ctypes.c_int64 * MAX_DIM), ("L", ctypes.c_double * MAX_DIM),
                ("growth", ctypes.c_double), ("periods", ctypes.c_double * (MAX_DIM * MAX_DIM))]


class Stats(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("n_step1", ctypes.c_int64),
                ("n_box", ctypes.c_int64), ("n_out", ctypes.c_int64),
                ("n_step2", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("oracle not built: run __graft_entry__.build() "
                               "or python oracle/build.py")
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        dp, ip, i64p = P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_int64)
        L.vto_validate.argtypes = [P(Problem), ctypes.c_int64, dp, dp]
        L.vto_choose_tau.argtypes = [P(Problem), ctypes.c_int64, dp]
        L.vto_choose_tau.restype = ctypes.c_double
        L.vto_cost_model.argtypes = [P(Problem), ctypes.c_int64, dp, ctypes.c_double]
        L.vto_cost_model.restype = ctypes.c_double
        L.vto_v0_fraction.argtypes = [ctypes.c_int64]
        L.vto_v0_fraction.restype = ctypes.c_double
        L.vto_tessellate.argtypes = [P(Problem), ctypes.c_int64, dp, dp, ctypes.c_double,
                                     ctypes.c_int, ip, dp, P(Stats)]
        L.vto_brute.argtypes = [P(Problem), ctypes.c_int64, dp, dp, ctypes.c_int, ip, dp]
        L.vto_label_points.argtypes = [P(Problem), ctypes.c_int64, dp, dp, ctypes.c_int64,
                                       i64p, ctypes.c_int, ip, dp]
        L.vto_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def problem(n, L, kind=VORONOI, periodic=True, growth=1.0, periods=None):
    """Problem statement: n voxels and lengths L per axis (1 to 6 entries).
    periods (optional, d x d, row i = period vector L_i): general periodic
    cell (App. A); L is then ignored and the boundaries are periodic."""
    n = list(n)
    L = list(L)
    if len(n) != len(L) or not 1 <= len(n) <= MAX_DIM:
        raise ValueError(f"n and L must both have 1 to {MAX_DIM} entries")
    p = Problem()
    p.ndim = len(n)
    p.kind = int(kind)
    p.periodic = 1 if periodic else 0
    for a in range(MAX_DIM):
        p.n[a] = int(n[a]) if a < len(n) else 1
        p.L[a] = float(L[a]) if a < len(L) else 1.0
    p.growth = float(growth)
    if periods is not None:
        P = np.asarray(periods, dtype=np.float64)
        if P.shape != (len(n), len(n)):
            raise ValueError("periods must be ndim x ndim")
        p.lattice = 1
        p.periodic = 1
        for k, v in enumerate(P.ravel()):
            p.periods[k] = float(v)
    return p


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _prep(p, coords, param):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    if coords.ndim != 2 or coords.shape[1] != p.ndim:
        raise ValueError("coords must be [nsites, ndim]")
    if param is not None:
        param = np.ascontiguousarray(param, dtype=np.float64)
        if param.shape != (coords.shape[0],):
            raise ValueError("param must be [nsites]")
    return coords, param


def shape_of(p):
    """numpy shape of the label image (slowest axis first)."""
    return tuple(p.n[a] for a in reversed(range(p.ndim)))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned status {code}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise OracleError(rc)


def validate(p, coords, param=None):
    coords, param = _prep(p, coords, param)
    return lib().vto_validate(ctypes.byref(p), coords.shape[0], _dptr(coords), _dptr(param))


def choose_tau(p, coords, param=None):
    coords, param = _prep(p, coords, param)
    return lib().vto_choose_tau(ctypes.byref(p), coords.shape[0], _dptr(param))


def cost_model(p, nsites, param=None, tau=float("nan")):
    if param is not None:
        param = np.ascontiguousarray(param, dtype=np.float64)
    return lib().vto_cost_model(ctypes.byref(p), int(nsites), _dptr(param), float(tau))


def v0_fraction(nsites):
    return lib().vto_v0_fraction(int(nsites))


def tessellate(p, coords, param=None, tau=float("nan"), nthreads=0, want_keys=False):
    """Two-step ball algorithm; returns (labels, keys or None, stats dict)."""
    coords, param = _prep(p, coords, param)
    labels = np.empty(shape_of(p), dtype=np.int32)
    keys = np.empty(shape_of(p), dtype=np.float64) if want_keys else None
    st = Stats()
    rc = lib().vto_tessellate(ctypes.byref(p), coords.shape[0], _dptr(coords), _dptr(param),
                              float(tau), int(nthreads),
                              labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              _dptr(keys), ctypes.byref(st))
    _check(rc)
    stats = dict(tau=st.tau, n_step1=st.n_step1, n_box=st.n_box, n_out=st.n_out,
                 n_step2=st.n_step2)
    return labels, keys, stats


def brute(p, coords, param=None, nthreads=0, want_keys=False):
    coords, param = _prep(p, coords, param)
    labels = np.empty(shape_of(p), dtype=np.int32)
    keys = np.empty(shape_of(p), dtype=np.float64) if want_keys else None
    rc = lib().vto_brute(ctypes.byref(p), coords.shape[0], _dptr(coords), _dptr(param),
                         int(nthreads), labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         _dptr(keys))
    _check(rc)
    return (labels, keys) if want_keys else labels


def label_points(p, coords, param, vox, nthreads=0):
    """Brute force at voxel indices vox [npts, ndim]; returns (labels, keys)."""
    coords, param = _prep(p, coords, param)
    vox = np.asarray(vox, dtype=np.int64)
    v3 = np.zeros((vox.shape[0], MAX_DIM), dtype=np.int64)
    v3[:, :vox.shape[1]] = vox
    labels = np.empty(vox.shape[0], dtype=np.int32)
    keys = np.empty(vox.shape[0], dtype=np.float64)
    rc = lib().vto_label_points(ctypes.byref(p), coords.shape[0], _dptr(coords), _dptr(param),
                                v3.shape[0], v3.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                int(nthreads), labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                _dptr(keys))
    _check(rc)
    return labels, keys


def max_threads():
    return lib().vto_max_threads()


def r0_voronoi(ndim, V, nsites):
    """Ball radius of eq. v0_3d: v0 = V (1 - N^(-1/(N-1))), v0 = omega_d r0^d."""
    v0 = v0_fraction(nsites) * V
    omega = math.pi ** (ndim / 2) / math.gamma(ndim / 2 + 1)
    return (v0 / omega) ** (1.0 / ndim)
