"""Leapfrog sessions: particle state resident on the GPU, stepped through libtfmm.

A Session keeps positions, velocities, masses and forces in device tensors and
one libtfmm tree; every step is a kick-drift-kick leapfrog step executed by
the library (tfmm_leapfrog), so the state never leaves the GPU between steps.
With the conserving (realigned) force every pair force is central and
antisymmetric, so the discrete leapfrog map conserves angular momentum up to
roundoff; with the standard expansion the spurious torques of Eq.
total_torque make it drift.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from .api import PRECISIONS, VARIANTS, Context, Tree, _check_vec
from ._lib import Params


class Session:
    def __init__(self, ctx: Context, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor, p: int = 4,
                 theta: float = 0.5, eps: float = 1e-3, variant: str = "conserving",
                 precision: str = "mixed32", n_leaf: int = 64, G: float = 1.0,
                 stream: Optional[torch.cuda.Stream] = None):
        n = int(mass.shape[0])
        for name, t, shape in (("pos", pos, (n, 3)), ("vel", vel, (n, 3)), ("mass", mass, (n,))):
            _check_vec(t, name, shape)
        self.ctx = ctx
        self.n = n
        self.stream = stream
        self.pos = pos.clone()
        self.vel = vel.clone()
        self.mass = mass.clone()
        self.force = torch.zeros_like(self.pos)
        self.params = dict(p=int(p), theta=float(theta), eps=float(eps), variant=variant, precision=precision,
                           G=float(G))
        self.n_leaf = int(n_leaf)
        self.step_count = 0
        self.time = 0.0
        with self._stream_ctx():
            self.tree = Tree(ctx, self.pos, self.mass, n_leaf=self.n_leaf)
        self._force_valid = False

    def _stream_ctx(self):
        return torch.cuda.stream(self.stream) if self.stream is not None else torch.cuda.stream(
            torch.cuda.current_stream(self.pos.device))

    def _prm(self) -> Params:
        q = self.params
        return Params(q["p"], q["theta"], q["eps"], q["G"], VARIANTS[q["variant"]], PRECISIONS[q["precision"]])

    def step(self, dt: float, nsteps: int = 1) -> None:
        """Advance nsteps kick-drift-kick steps of size dt (synchronising)."""
        prm = self._prm()
        with self._stream_ctx():
            s = torch.cuda.current_stream(self.pos.device).cuda_stream
            self.ctx.check(self.ctx.lib.tfmm_leapfrog(
                self.tree.handle, ctypes.byref(prm), self.pos.data_ptr(), self.vel.data_ptr(),
                self.mass.data_ptr(), self.force.data_ptr(), float(dt), int(nsteps), int(self._force_valid), s))
        self._force_valid = True
        self.step_count += int(nsteps)
        self.time += float(dt) * int(nsteps)

    def forces(self) -> torch.Tensor:
        """Forces at the current positions (evaluated if not yet known)."""
        if not self._force_valid:
            self.step(0.0, 0)
        return self.force

    def diagnostics(self) -> dict:
        """Net force / torque relative measures and the momenta P, L (FP64, on the GPU)."""
        f = self.forces()
        with self._stream_ctx():
            d = self.ctx.diagnostics(self.pos, self.mass, f, self.vel)
        return {"net_force": d[0:3], "net_torque": d[4:7], "P": d[8:11], "L": d[11:14], "mass": d[14],
                "com": d[15:18], "force_rel": float(d[18]), "torque_rel": float(d[19])}

    def energy(self) -> dict:
        """Kinetic, potential and total energy at the current state (FP64
        sums on the GPU): K = sum m v^2 / 2, W = sum m_a phi_a / 2 with phi from
        the library's potential output (an extra evaluation with the
        session's parameters; the resident forces are left as they are)."""
        self.forces()
        q = self.params
        with self._stream_ctx():
            f = torch.empty_like(self.pos)
            phi = torch.empty_like(self.mass)
            self.tree.evaluate(p=q["p"], theta=q["theta"], eps=q["eps"], variant=q["variant"],
                               precision=q["precision"], G=q["G"], out=f, pot=phi)
            K = 0.5 * float((self.mass * (self.vel * self.vel).sum(1)).sum())
            W = 0.5 * float((self.mass * phi).sum())
        return {"K": K, "W": W, "E": K + W}

    def snapshot(self, path) -> None:
        """Write the resident state and parameters to an .npz file."""
        torch.cuda.synchronize(self.pos.device)
        np.savez(path, pos=self.pos.cpu().numpy(), vel=self.vel.cpu().numpy(), mass=self.mass.cpu().numpy(),
                 step=self.step_count, time=self.time, n_leaf=self.n_leaf,
                 p=self.params["p"], theta=self.params["theta"], eps=self.params["eps"], G=self.params["G"],
                 variant=self.params["variant"], precision=self.params["precision"])

    @classmethod
    def restore(cls, ctx: Context, path, stream: Optional[torch.cuda.Stream] = None) -> "Session":
        z = np.load(path, allow_pickle=False)
        dev = torch.device("cuda", ctx.device)
        s = cls(ctx, torch.from_numpy(z["pos"]).to(dev), torch.from_numpy(z["vel"]).to(dev),
                torch.from_numpy(z["mass"]).to(dev), p=int(z["p"]), theta=float(z["theta"]), eps=float(z["eps"]),
                variant=str(z["variant"]), precision=str(z["precision"]), n_leaf=int(z["n_leaf"]),
                G=float(z["G"]), stream=stream)
        s.step_count = int(z["step"])
        s.time = float(z["time"])
        return s

    def close(self) -> None:
        if getattr(self, "tree", None) is not None:
            self.tree.close()
            self.tree = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint_bytes(n: int, p: int, n_leaf: int = 64, precision: str = "mixed32") -> int:
    """Device bytes a session of n particles needs: the tree plus the resident state."""
    lib = _lib.load()
    return int(lib.tfmm_footprint_bytes(int(n), int(p), int(n_leaf), PRECISIONS[precision])) + 4 * 24 * int(n)
