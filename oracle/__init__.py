"""Plain FP64 CPU oracle for the torque-free FMM force evaluation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark use it; the solver package never imports it and
shares no code with it.  The arithmetic lives in ``oracle.c`` (built into
``liboracle.so`` by ``oracle/build.py``); this module marshals numpy arrays.

Contents (paper: Korobkin et al., arXiv:2107.07166):

* ``direct``          -- O(N^2) softened direct sum (gradient of Eq. jia).
* ``series``          -- univariate Taylor coefficients of (c0+c1 t+c2 t^2)^alpha,
                         the degree-n parts of Eq. taylor along R + t*delta.
* ``pair_far`` / ``cluster_far`` -- truncated far-field pair accelerations,
                         standard (gradient of the truncated Eq. taylor) and
                         conserving (Eq. realign with the projection scalar
                         truncated at degree p-1, or at a higher degree K).
* ``Tree``            -- keys, stable order, octree, centres of mass, r_max
                         (Eq. mac_criterion), mutual walk, and FMM forces on any
                         subset of particles.
* ``diagnostics``     -- net force and net torque (Eqs. netforce, total_torque).
"""

from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_LIB_PATH = _HERE / "liboracle.so"

STANDARD = 0
CONSERVING = 1
CONSERVING_R2 = 2  # zeroth order, realigned by magnitude (Eq. realign2); p must be 1
VARIANTS = {"standard": STANDARD, "conserving": CONSERVING, "conserving_r2": CONSERVING_R2}

_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_i32 = ctypes.c_int
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(str(_LIB_PATH))
    lib.orc_direct.argtypes = [_i64, _vp, _vp, _d, _d, _vp, _vp]
    lib.orc_series.argtypes = [_d, _d, _d, _d, _i32, _vp]
    lib.orc_pair_far.argtypes = [_vp, _vp, _vp, _d, _i32, _i32, _d, _i32, _vp, _vp]
    lib.orc_cluster_far.argtypes = [_i64, _vp, _vp, _i64, _vp, _vp, _vp, _i32, _i32, _d, _i32, _vp, _vp]
    lib.orc_tree_build.argtypes = [_i64, _vp, _vp, _i64, _d]
    lib.orc_tree_build.restype = _vp
    lib.orc_tree_free.argtypes = [_vp]
    lib.orc_tree_free.restype = None
    lib.orc_tree_sizes.argtypes = [_vp, _vp]
    lib.orc_tree_sizes.restype = None
    lib.orc_tree_bbox.argtypes = [_vp, _vp]
    lib.orc_tree_bbox.restype = None
    lib.orc_tree_keys.argtypes = [_vp, _vp, _vp]
    lib.orc_tree_keys.restype = None
    lib.orc_tree_nodes.argtypes = [_vp] * 11
    lib.orc_tree_nodes.restype = None
    lib.orc_tree_lists.argtypes = [_vp, _vp, _vp]
    lib.orc_tree_lists.restype = None
    lib.orc_fmm_forces.argtypes = [_vp, _i32, _i32, _d, _d, _i32, _i64, _vp, _vp, _vp]
    lib.orc_diagnostics.argtypes = [_i64, _vp, _vp, _vp, _vp, _vp]
    lib.orc_set_threads.argtypes = [_i32]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def set_threads(n: int) -> int:
    """Set the OpenMP thread count (n <= 0 keeps it); returns the count in use."""
    return int(_load().orc_set_threads(int(n)))


def direct(pos, mass, eps=0.0, G=1.0, with_potential=False):
    """Softened direct sum: F_a = -G m_a sum_b m_b (X_a-X_b)(|X_a-X_b|^2+eps^2)^(-3/2)."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    mass = _f64(mass)
    n = len(mass)
    f = np.empty((n, 3))
    pot = np.empty(n) if with_potential else None
    rc = lib.orc_direct(n, _ptr(pos), _ptr(mass), float(eps), float(G), _ptr(f), _ptr(pot))
    if rc:
        raise ValueError("orc_direct failed")
    return (f, pot) if with_potential else f


def series(c0, c1, c2, alpha, nmax):
    """Coefficients w_0..w_nmax of (c0 + c1 t + c2 t^2)^alpha."""
    w = np.empty(nmax + 1)
    if _load().orc_series(float(c0), float(c1), float(c2), float(alpha), int(nmax), _ptr(w)):
        raise ValueError("orc_series: c0 must be > 0 and nmax >= 0")
    return w


def pair_far(R, x, y, mb, p, eps, variant="standard", scalar_degree=0):
    """Truncated far-field acceleration (G=1) of a at Z_A+x due to b at Z_B+y.

    scalar_degree: degree K of the conserving projection scalar (0 = p-1)."""
    R, x, y = _f64(R), _f64(x), _f64(y)
    acc = np.empty(3)
    pot = np.empty(1)
    rc = _load().orc_pair_far(_ptr(R), _ptr(x), _ptr(y), float(mb), int(p), int(scalar_degree),
                              float(eps), VARIANTS[variant], _ptr(acc), _ptr(pot))
    if rc:
        raise ValueError("orc_pair_far: bad arguments")
    return acc, float(pot[0])


def cluster_far(Xt, ZA, Ys, ms, ZB, p, eps, variant="standard", scalar_degree=0):
    """Far-field accelerations (G=1) on targets Xt (node centre ZA) from sources Ys, ms (centre ZB)."""
    Xt = _f64(Xt, (-1, 3))
    Ys = _f64(Ys, (-1, 3))
    ms = _f64(ms)
    ZA, ZB = _f64(ZA), _f64(ZB)
    acc = np.empty((len(Xt), 3))
    pot = np.empty(len(Xt))
    rc = _load().orc_cluster_far(len(Xt), _ptr(Xt), _ptr(ZA), len(Ys), _ptr(Ys), _ptr(ms),
                                 _ptr(ZB), int(p), int(scalar_degree), float(eps), VARIANTS[variant],
                                 _ptr(acc), _ptr(pot))
    if rc:
        raise ValueError("orc_cluster_far: bad arguments")
    return acc, pot


def diagnostics(pos, mass, force, vel=None):
    """Net force / torque / momenta (see orc_diagnostics for the 20 slots)."""
    pos = _f64(pos, (-1, 3))
    force = _f64(force, (-1, 3))
    mass = _f64(mass)
    vel = None if vel is None else _f64(vel, (-1, 3))
    out = np.empty(20)
    if _load().orc_diagnostics(len(mass), _ptr(pos), _ptr(vel), _ptr(mass), _ptr(force), _ptr(out)):
        raise ValueError("orc_diagnostics failed")
    return out


class Tree:
    """Oracle octree + mutual walk for one particle set (n_leaf, theta fixed)."""

    def __init__(self, pos, mass, n_leaf=64, theta=0.5):
        lib = _load()
        self._pos = _f64(pos, (-1, 3))
        self._mass = _f64(mass)
        self.n_leaf = int(n_leaf)
        self.theta = float(theta)
        h = lib.orc_tree_build(len(self._mass), _ptr(self._pos), _ptr(self._mass),
                               self.n_leaf, self.theta)
        if not h:
            raise ValueError("orc_tree_build failed (bad arguments or out of memory)")
        self._h = ctypes.c_void_p(h)
        sz = np.empty(4, dtype=np.int64)
        lib.orc_tree_sizes(self._h, _ptr(sz))
        self.n, self.n_nodes, self.n_m2l, self.n_p2p = (int(v) for v in sz)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_tree_free(h)
            self._h = None

    def bbox(self):
        out = np.empty(5)
        _load().orc_tree_bbox(self._h, _ptr(out))
        return out

    def keys(self):
        """(keys in original order as uint64, order: sorted position -> original index)."""
        k = np.empty(self.n, dtype=np.uint64)
        o = np.empty(self.n, dtype=np.int64)
        _load().orc_tree_keys(self._h, _ptr(k), _ptr(o))
        return k, o

    def nodes(self):
        nn = self.n_nodes
        d = dict(level=np.empty(nn, np.int32), prefix=np.empty(nn, np.uint64),
                 first=np.empty(nn, np.int64), count=np.empty(nn, np.int64),
                 child_first=np.empty(nn, np.int64), nchild=np.empty(nn, np.int32),
                 parent=np.empty(nn, np.int64), mass=np.empty(nn), com=np.empty((nn, 3)),
                 rmax=np.empty(nn))
        _load().orc_tree_nodes(self._h, *(_ptr(d[k]) for k in (
            "level", "prefix", "first", "count", "child_first", "nchild", "parent",
            "mass", "com", "rmax")))
        return d

    def lists(self):
        """(far pairs, near pairs) as int64 arrays of shape (k, 2), lower index first."""
        m = np.empty((self.n_m2l, 2), dtype=np.int64)
        p = np.empty((self.n_p2p, 2), dtype=np.int64)
        _load().orc_tree_lists(self._h, _ptr(m), _ptr(p))
        return m, p

    def forces(self, p, eps, variant="standard", G=1.0, targets=None, with_potential=False,
               scalar_degree=0):
        """FMM forces (and optionally potentials) on `targets` (original indices) or all.

        scalar_degree: degree K of the conserving projection scalar (0 = p-1)."""
        lib = _load()
        tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
        nt = self.n if tg is None else len(tg)
        f = np.empty((nt, 3))
        pot = np.empty(nt) if with_potential else None
        rc = lib.orc_fmm_forces(self._h, int(p), int(scalar_degree), float(eps), float(G), VARIANTS[variant],
                                nt, _ptr(tg), _ptr(f), _ptr(pot))
        if rc:
            raise ValueError(f"orc_fmm_forces failed ({rc})")
        return (f, pot) if with_potential else f


def lib_path() -> str:
    return os.fspath(_LIB_PATH)
