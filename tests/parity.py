"""Shared gates of the GPU parity tests (not a test module).

Every force comparison checks two things against the FP64 oracle:

* the rms over particles of |F_gpu - F_ref| / |F_ref| (the error measure of
  the paper's distance test, Sec. 4), against 1e-12 (FP64 path) and 2e-6
  (mixed path: FP32 near and far fields, FP64 accumulation);
* the largest per-particle |F_gpu - F_ref| / |F_ref|, against 1e-12 (FP64)
  and 3e-4 (mixed).  In the mixed path every particle enters the FP32
  kernels as its offset from its leaf's centre of mass, rounded once, so a
  pair at separation r in a leaf of radius r_leaf carries a relative error
  of about 2^-24 r_leaf / sqrt(r^2 + eps^2).  With eps = 1e-3 that stays
  below ~1e-5 (largest measured on the tree workloads: 1.1e-5); the
  two-body setup of the distance test has eps = 0 and leaves of radius 1,
  and its closest pairs reach 4.8e-5.  The FP64 path measures at most
  6e-14.  A wrong leaf, list entry or expansion term gives 1e-3 or more.

Net force |sum F| / sum |F| (Eq. netforce): 1e-14 (FP64; measured <= 4e-16)
and 2e-7 (mixed; measured <= 1.5e-8): the two directions of every pair are
computed separately, each with its own rounding.  Net torque of the
realigned variants (Eq. total_torque, Sec. 3.2): 1e-14 (FP64; measured
<= 2.3e-16) and 1e-6 (mixed; measured <= 7.3e-9).
"""

import numpy as np

TOL_RMS = {"fp64": 1e-12, "mixed32": 2e-6}
TOL_MAX = {"fp64": 1e-12, "mixed32": 3e-4}
TOL_NETFORCE = {"fp64": 1e-14, "mixed32": 2e-7}
TOL_TORQUE = {"fp64": 1e-14, "mixed32": 1e-6}


def rel_errors(f, ref):
    f = np.asarray(f, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.sqrt(((f - ref) ** 2).sum(1) / (ref ** 2).sum(1))


def erms(f, ref):
    return float(np.sqrt(np.mean(rel_errors(f, ref) ** 2)))


def gate(f, ref, prec, what=""):
    """Assert the rms and max gates; returns (rms, max) for reporting."""
    e = rel_errors(f, ref)
    rms = float(np.sqrt(np.mean(e ** 2)))
    mx = float(e.max()) if len(e) else 0.0
    print(f"  parity {what} {prec}: rms {rms:.3e} max {mx:.3e} over {len(e)} particles", flush=True)
    assert rms <= TOL_RMS[prec], (what, prec, "rms", rms)
    assert mx <= TOL_MAX[prec], (what, prec, "max", mx, int(np.argmax(e)))
    return rms, mx


def gate_momenta(diag, prec, variant, what=""):
    """Net force for every variant, net torque for the realigned ones."""
    print(f"  momenta {what} {variant} {prec}: net force {diag[18]:.3e} net torque {diag[19]:.3e}", flush=True)
    assert diag[18] <= TOL_NETFORCE[prec], (what, prec, variant, "net force", diag[18])
    if variant in ("conserving", "conserving_r2"):
        assert diag[19] <= TOL_TORQUE[prec], (what, prec, variant, "net torque", diag[19])
