"""Python binding of libtfmm on torch tensors (argument marshalling only).

Every step of the force evaluation runs in the HIP library; torch provides
device memory (the caller's tensors) and the current HIP stream.

    import torch
    from paper_2107_07166_amd import api
    f = api.evaluate_forces(pos, mass, p=4, theta=0.5, eps=1e-3,
                            variant="conserving", precision="mixed32")

`pos` is an (N, 3) float64 tensor on the GPU, `mass` (N,) float64; the result
is the (N, 3) float64 force F_a = G m_a a_a in the input order.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import Params, TfmmError

VARIANTS = {"standard": _lib.STANDARD, "conserving": _lib.CONSERVING, "conserving_r2": _lib.CONSERVING_R2}
PRECISIONS = {"fp64": _lib.FP64, "mixed32": _lib.MIXED32}


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_vec(t: torch.Tensor, name: str, shape) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Context:
    """A libtfmm context: one device, an optional device-memory budget."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.lib = _lib.load()
        self.device = int(device)
        h = ctypes.c_void_p()
        rc = self.lib.tfmm_ctx_create(self.device, int(budget_bytes), ctypes.byref(h))
        if rc != _lib.OK:
            raise TfmmError(rc, f"tfmm_ctx_create(device={device}) failed")
        self.handle = h
        self._trees = set()

    def check(self, rc: int) -> None:
        if rc != _lib.OK:
            msg = self.lib.tfmm_last_error(self.handle)
            raise TfmmError(rc, msg.decode() if msg else "")

    def bytes_in_use(self) -> int:
        return int(self.lib.tfmm_ctx_bytes_in_use(self.handle))

    def bytes_held(self) -> int:
        """Device bytes held, including released blocks kept for reuse."""
        return int(self.lib.tfmm_ctx_bytes_held(self.handle))

    def set_budget(self, budget_bytes: int) -> None:
        """Device-memory budget for later allocations (0 = no limit)."""
        self.check(self.lib.tfmm_ctx_set_budget(self.handle, int(budget_bytes)))

    def trim(self) -> None:
        """Give the released blocks kept for reuse back to the device."""
        self.check(self.lib.tfmm_ctx_trim(self.handle))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            for t in list(self._trees):
                t.close()
            self.check(self.lib.tfmm_ctx_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def diagnostics(self, pos, mass, force, vel=None) -> np.ndarray:
        n = mass.shape[0]
        _check_vec(pos, "pos", (n, 3))
        _check_vec(mass, "mass", (n,))
        _check_vec(force, "force", (n, 3))
        if vel is not None:
            _check_vec(vel, "vel", (n, 3))
        out = np.zeros(20)
        self.check(self.lib.tfmm_momentum_diagnostics(
            self.handle, n, pos.data_ptr(), None if vel is None else vel.data_ptr(), mass.data_ptr(),
            force.data_ptr(), _stream_handle(pos.device), out.ctypes.data_as(ctypes.c_void_p)))
        return out


def _offsets(offsets, n: int) -> np.ndarray:
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or off.size < 2 or off[-1] != n:
        raise ValueError("offsets must be 1-D, n_sets + 1 values ending at the particle count")
    return off


class Tree:
    """Octree of one particle set (or a forest of independent sets), with its
    walk and expansions cached."""

    def __init__(self, ctx: Context, pos: torch.Tensor, mass: torch.Tensor, n_leaf: int = 64, offsets=None):
        """offsets: None for one particle set, else the n_sets + 1 boundaries
        of a forest (set k is particles offsets[k] .. offsets[k+1]-1)."""
        n = int(mass.shape[0])
        _check_vec(pos, "pos", (n, 3))
        _check_vec(mass, "mass", (n,))
        self.ctx = ctx
        self.n = n
        self.n_leaf = int(n_leaf)
        self.device = pos.device
        h = ctypes.c_void_p()
        if offsets is None:
            self.n_sets = 1
            ctx.check(ctx.lib.tfmm_build_tree(ctx.handle, n, pos.data_ptr(), mass.data_ptr(), self.n_leaf,
                                              _stream_handle(pos.device), ctypes.byref(h)))
        else:
            off = _offsets(offsets, n)
            self.n_sets = int(off.size - 1)
            ctx.check(ctx.lib.tfmm_build_forest(ctx.handle, self.n_sets, off.ctypes.data_as(ctypes.c_void_p),
                                                pos.data_ptr(), mass.data_ptr(), self.n_leaf,
                                                _stream_handle(pos.device), ctypes.byref(h)))
        self.handle = h
        ctx._trees.add(self)

    def rebuild(self, pos: torch.Tensor, mass: torch.Tensor, offsets=None) -> None:
        """Rebuild for new positions; the particle count may change (buffers
        are grow-only).  offsets: as in the constructor (None: one set)."""
        n = int(mass.shape[0])
        _check_vec(pos, "pos", (n, 3))
        _check_vec(mass, "mass", (n,))
        if offsets is None:
            self.ctx.check(self.ctx.lib.tfmm_tree_rebuild(self.handle, n, pos.data_ptr(), mass.data_ptr(),
                                                          _stream_handle(pos.device)))
            self.n_sets = 1
        else:
            off = _offsets(offsets, n)
            self.ctx.check(self.ctx.lib.tfmm_forest_rebuild(self.handle, int(off.size - 1),
                                                            off.ctypes.data_as(ctypes.c_void_p), pos.data_ptr(),
                                                            mass.data_ptr(), _stream_handle(pos.device)))
            self.n_sets = int(off.size - 1)
        self.n = n

    def walk(self, theta: float) -> None:
        self.ctx.check(self.ctx.lib.tfmm_tree_walk(self.handle, float(theta), _stream_handle(self.device)))

    def evaluate(self, p: int = 4, theta: float = 0.5, eps: float = 1e-3, variant: str = "conserving",
                 precision: str = "mixed32", G: float = 1.0,
                 out: Optional[torch.Tensor] = None, pot: Optional[torch.Tensor] = None,
                 scalar_degree: int = 0) -> torch.Tensor:
        """Forces into `out` (n x 3); if `pot` (n) is given, also G times the
        potential at every particle (standard expansion for the far field).
        scalar_degree: degree of the conserving projection scalar (0 = p - 1)."""
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        _check_vec(out, "out", (self.n, 3))
        pot_ptr = None
        if pot is not None:
            _check_vec(pot, "pot", (self.n,))
            pot_ptr = pot.data_ptr()
        prm = Params(int(p), float(theta), float(eps), float(G), VARIANTS[variant], PRECISIONS[precision],
                     int(scalar_degree))
        self.ctx.check(self.ctx.lib.tfmm_evaluate_forces(self.handle, ctypes.byref(prm), out.data_ptr(), pot_ptr,
                                                         _stream_handle(self.device)))
        return out

    def evaluate_forest(self, thetas, p: int = 4, eps: float = 1e-3, variant: str = "conserving",
                        precision: str = "mixed32", G: float = 1.0, out: Optional[torch.Tensor] = None,
                        pot: Optional[torch.Tensor] = None, scalar_degree: int = 0) -> torch.Tensor:
        """evaluate() with one theta per set of the forest (tfmm_evaluate_forest)."""
        th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64))
        if th.shape != (self.n_sets,):
            raise ValueError(f"thetas must hold one value per set ({self.n_sets})")
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        _check_vec(out, "out", (self.n, 3))
        pot_ptr = None
        if pot is not None:
            _check_vec(pot, "pot", (self.n,))
            pot_ptr = pot.data_ptr()
        prm = Params(int(p), float(th[0]), float(eps), float(G), VARIANTS[variant], PRECISIONS[precision],
                     int(scalar_degree))
        self.ctx.check(self.ctx.lib.tfmm_evaluate_forest(self.handle, ctypes.byref(prm),
                                                         th.ctypes.data_as(ctypes.c_void_p), out.data_ptr(),
                                                         pot_ptr, _stream_handle(self.device)))
        return out

    def info(self) -> dict:
        a = np.zeros(8, dtype=np.int64)
        self.ctx.check(self.ctx.lib.tfmm_tree_info(self.handle, a.ctypes.data_as(ctypes.c_void_p)))
        keys = ("n", "nodes", "leaves", "max_level", "far_pairs", "near_pairs", "near_interactions",
                "far_directed")
        return {k: int(v) for k, v in zip(keys, a)}

    def export(self) -> dict:
        inf = self.info()
        n, nn = self.n, inf["nodes"]
        d = dict(keys=np.empty(n, np.uint64), order=np.empty(n, np.int32), level=np.empty(nn, np.int32),
                 prefix=np.empty(nn, np.uint64), first=np.empty(nn, np.int32), count=np.empty(nn, np.int32),
                 child_first=np.empty(nn, np.int32), nchild=np.empty(nn, np.int32),
                 parent=np.empty(nn, np.int32), com=np.empty((nn, 3)), mass=np.empty(nn),
                 rmax=np.empty(nn))
        ptr = {k: v.ctypes.data_as(ctypes.c_void_p) for k, v in d.items()}
        self.ctx.check(self.ctx.lib.tfmm_tree_export(
            self.handle, ptr["keys"], ptr["order"], ptr["level"], ptr["prefix"], ptr["first"], ptr["count"],
            ptr["child_first"], ptr["nchild"], ptr["parent"], ptr["com"], ptr["mass"], ptr["rmax"]))
        return d

    def lists(self):
        inf = self.info()
        far = np.empty((max(inf["far_pairs"], 0), 2), np.int32)
        near = np.empty((max(inf["near_pairs"], 0), 2), np.int32)
        self.ctx.check(self.ctx.lib.tfmm_lists_export(self.handle, far.ctypes.data_as(ctypes.c_void_p),
                                                      near.ctypes.data_as(ctypes.c_void_p)))
        return far, near

    def set_timing(self, enable: bool = True) -> None:
        self.ctx.check(self.ctx.lib.tfmm_tree_set_timing(self.handle, int(bool(enable))))

    def phase_times(self) -> dict:
        """Average device times (ms) of the timed evaluations and rebuilds."""
        a = np.zeros(10)
        self.ctx.check(self.ctx.lib.tfmm_tree_phase_times(self.handle, a.ctypes.data_as(ctypes.c_void_p)))
        return dict(zip(("m2l", "p2p", "l2l", "l2p", "moments", "total", "rebuild", "walk", "walk_passes",
                         "interaction"), a.tolist()))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            self.ctx.lib.tfmm_tree_destroy(self.handle)
            self.handle = None
            self.ctx._trees.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Optional[Context] = None


def default_context(device: int = 0) -> Context:
    global _default_ctx
    if _default_ctx is None or _default_ctx.device != device:
        _default_ctx = Context(device)
    return _default_ctx


def evaluate_forces(pos: torch.Tensor, mass: torch.Tensor, p: int = 4, theta: float = 0.5, eps: float = 1e-3,
                    variant: str = "conserving", precision: str = "mixed32", n_leaf: int = 64, G: float = 1.0,
                    ctx: Optional[Context] = None) -> torch.Tensor:
    """Build the tree and evaluate the FMM forces in one call."""
    ctx = ctx or default_context(pos.device.index or 0)
    t = Tree(ctx, pos, mass, n_leaf=n_leaf)
    try:
        return t.evaluate(p=p, theta=theta, eps=eps, variant=variant, precision=precision, G=G)
    finally:
        torch.cuda.current_stream(pos.device).synchronize()
        t.close()


def evaluate_forces_oneshot(pos: torch.Tensor, mass: torch.Tensor, p: int = 4, theta: float = 0.5,
                            eps: float = 1e-3, variant: str = "conserving", precision: str = "mixed32",
                            n_leaf: int = 64, G: float = 1.0, ctx: Optional[Context] = None,
                            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Build, evaluate and destroy a tree in one library call
    (tfmm_evaluate_forces_oneshot; synchronising)."""
    ctx = ctx or default_context(pos.device.index or 0)
    n = int(mass.shape[0])
    _check_vec(pos, "pos", (n, 3))
    _check_vec(mass, "mass", (n,))
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    _check_vec(out, "out", (n, 3))
    prm = Params(int(p), float(theta), float(eps), float(G), VARIANTS[variant], PRECISIONS[precision])
    ctx.check(ctx.lib.tfmm_evaluate_forces_oneshot(ctx.handle, n, pos.data_ptr(), mass.data_ptr(), int(n_leaf),
                                                   ctypes.byref(prm), out.data_ptr(),
                                                   _stream_handle(pos.device)))
    return out


def momentum_diagnostics(pos, mass, force, vel=None, ctx: Optional[Context] = None) -> np.ndarray:
    ctx = ctx or default_context(pos.device.index or 0)
    return ctx.diagnostics(pos, mass, force, vel)


def footprint_bytes(n: int, p: int, n_leaf: int = 64, precision: str = "mixed32") -> int:
    return int(_lib.load().tfmm_footprint_bytes(int(n), int(p), int(n_leaf), PRECISIONS[precision]))
