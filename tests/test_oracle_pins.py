"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Paper: Korobkin et al., "Conservation of Angular Momentum in the Fast
Multipole Method", arXiv:2107.07166.  Each test names the passage it checks.
None of these tests retypes the oracle's own formula: they compare it with
library special functions (scipy Gegenbauer polynomials), with sympy's
symbolic Taylor series of the defining expressions, with the paper's printed
closed forms (the D tensors, Eq. potential, Eq. g_acc_BtoA, Eq. aaB1), with
the direct sum, and with invariants (momentum balance, zero torque, pair
coverage, convergence).
"""

import math

import numpy as np
import pytest
import scipy.special as sps
import sympy as sp

import oracle
from paper_2107_07166_amd.generators import plummer, uniform_ball


def _rng(seed=1):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# Degree-n parts of Eq. taylor along R + t*delta: Gegenbauer generating function
# (1 - 2 x h + h^2)^(-lam) = sum_n C_n^(lam)(x) h^n.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("alpha,lam", [(-0.5, 0.5), (-1.5, 1.5)])
def test_series_matches_gegenbauer(alpha, lam):
    rng = _rng(2)
    for _ in range(50):
        R = rng.normal(size=3)
        d = rng.normal(size=3) * rng.uniform(0.05, 0.9)
        eps = rng.choice([0.0, 1e-3, 0.3])
        c0 = R @ R + eps * eps
        c1 = 2.0 * (R @ d)
        c2 = d @ d
        w = oracle.series(c0, c1, c2, alpha, 8)
        h = math.sqrt(c2 / c0)
        x = -c1 / (2.0 * math.sqrt(c0 * c2))
        ref = np.array([c0 ** alpha * sps.eval_gegenbauer(n, lam, x) * h ** n for n in range(9)])
        np.testing.assert_allclose(w, ref, rtol=1e-12, atol=1e-14 * abs(ref[0]))


def test_series_sums_to_kernel_for_small_delta():
    # sum of all degree-n parts converges to the kernel itself (|delta| << |R|)
    R = np.array([1.0, 0.4, -0.2])
    d = np.array([0.01, -0.02, 0.015])
    c0, c1, c2 = R @ R, 2 * R @ d, d @ d
    w = oracle.series(c0, c1, c2, -1.5, 8)
    exact = ((R + d) @ (R + d)) ** -1.5
    assert abs(w.sum() - exact) < 1e-14 * exact


# ---------------------------------------------------------------------------
# Single pair, standard and conserving, against sympy's Taylor series of the
# defining expressions (Eq. taylor; Eq. realign with the projection scalar
# expanded in delta as in Eqs. nab-expansion / abnab-expansion, kept to
# degree p-1).
# ---------------------------------------------------------------------------
def _sympy_pair(R, dnum, eps, p):
    t = sp.Symbol("t")
    dx, dy, dz = sp.symbols("dx dy dz")
    Rs = [sp.Float(v, 30) for v in R]
    e2 = sp.Float(eps, 30) ** 2
    phi = -((Rs[0] + t * dx) ** 2 + (Rs[1] + t * dy) ** 2 + (Rs[2] + t * dz) ** 2 + e2) ** sp.Rational(-1, 2)
    Tp = sp.series(phi, t, 0, p + 1).removeO().subs(t, 1)
    grad = [sp.diff(Tp, v) for v in (dx, dy, dz)]
    sub = {dx: dnum[0], dy: dnum[1], dz: dnum[2]}
    a_std = np.array([-float(g.subs(sub)) for g in grad])
    pot = float(Tp.subs(sub))
    # projection scalar (a.u)/|u|^2 along delta -> t*delta, truncated at degree p-1
    tsub = {dx: t * dnum[0], dy: t * dnum[1], dz: t * dnum[2]}
    a_t = [-g.subs(tsub) for g in grad]
    u_t = [Rs[k] + t * dnum[k] for k in range(3)]
    scal = (a_t[0] * u_t[0] + a_t[1] * u_t[1] + a_t[2] * u_t[2]) / (u_t[0] ** 2 + u_t[1] ** 2 + u_t[2] ** 2)
    scal_p = float(sp.series(scal, t, 0, p).removeO().subs(t, 1))
    u = np.array(R) + np.array(dnum)
    a_cons = scal_p * u
    return a_std, a_cons, pot


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_pair_far_matches_sympy_taylor(p):
    rng = _rng(10 + p)
    for trial in range(3):
        R = rng.normal(size=3)
        R *= rng.uniform(1.0, 3.0) / np.linalg.norm(R)
        x = rng.normal(size=3) * 0.2
        y = rng.normal(size=3) * 0.2
        eps = [0.0, 1e-3, 0.2][trial]
        a_std, a_cons, pot = _sympy_pair(R, x - y, eps, p)
        acc_s, pot_s = oracle.pair_far(R, x, y, 1.0, p, eps, "standard")
        acc_c, _ = oracle.pair_far(R, x, y, 1.0, p, eps, "conserving")
        np.testing.assert_allclose(acc_s, a_std, rtol=1e-11, atol=1e-13 * np.linalg.norm(a_std))
        np.testing.assert_allclose(acc_c, a_cons, rtol=1e-11, atol=1e-13 * np.linalg.norm(a_cons))
        assert abs(pot_s - pot) <= 1e-12 * abs(pot)
        # conserving pair force is central: parallel to u = X_a - Y_b = R + delta
        u = R + x - y
        assert np.linalg.norm(np.cross(acc_c, u)) <= 1e-13 * np.linalg.norm(acc_c) * np.linalg.norm(u)


# ---------------------------------------------------------------------------
# The paper's printed closed forms at eps = 0.
# ---------------------------------------------------------------------------
def _D_tensors(R):
    """Eqs. D, Di, Dij, Dijk, Dijkl: derivatives of -1/R as printed."""
    R = np.asarray(R, float)
    r = np.linalg.norm(R)
    I = np.eye(3)
    D0 = -1.0 / r
    D1 = R / r ** 3
    D2 = (-3.0 * np.einsum("i,j->ij", R, R) + I * r ** 2) / r ** 5
    D3 = (15.0 * np.einsum("i,j,k->ijk", R, R, R)
          - 3.0 * r ** 2 * (np.einsum("ij,k->ijk", I, R) + np.einsum("jk,i->ijk", I, R)
                            + np.einsum("ik,j->ijk", I, R))) / r ** 7
    RR = np.einsum("i,j->ij", R, R)
    D4 = (-105.0 * np.einsum("i,j,k,l->ijkl", R, R, R, R)
          + 15.0 * r ** 2 * (np.einsum("ij,kl->ijkl", I, RR) + np.einsum("il,jk->ijkl", I, RR)
                             + np.einsum("ik,jl->ijkl", I, RR) + np.einsum("jl,ik->ijkl", I, RR)
                             + np.einsum("jk,il->ijkl", I, RR) + np.einsum("lk,ij->ijkl", I, RR))
          - 3.0 * r ** 4 * (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I)
                            + np.einsum("il,jk->ijkl", I, I))) / r ** 9
    return D0, D1, D2, D3, D4


def _two_clusters(seed, nb=40, na=7, dist=3.0, size=0.3):
    rng = _rng(seed)
    Ys = rng.normal(size=(nb, 3)) * size
    ms = rng.uniform(0.5, 1.5, nb)
    ZB = (ms[:, None] * Ys).sum(0) / ms.sum()
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    Xt = rng.normal(size=(na, 3)) * size + dist * direction
    ZA = Xt.mean(0)  # any expansion centre works for the targets
    return Xt, ZA, Ys, ms, ZB


def test_D_tensors_are_derivatives_of_minus_inverse_r():
    # The printed D tensors are successive derivatives of phi = -1/r
    # (fourth-order central differences of the next-lower printed tensor).
    R = np.array([0.9, -0.4, 0.7])
    D = _D_tensors(R)
    h = 1e-3
    I = np.eye(3)
    for i in range(3):
        f = [_D_tensors(R + k * h * I[i]) for k in (2, 1, -1, -2)]
        for n in range(4):
            fd = (-f[0][n] + 8 * f[1][n] - 8 * f[2][n] + f[3][n]) / (12 * h)
            ref = np.take(D[n + 1], i, axis=0)
            np.testing.assert_allclose(fd, ref, rtol=1e-8, atol=1e-9 * np.abs(D[n + 1]).max())


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_p4_standard_matches_eq_g_acc_BtoA(seed):
    """Eq. g_acc_BtoA (4th-order acceleration) with raw moments Q = sum m y y,
    H = -sum m y y y; only this reading of the printed moments makes Eq.
    potential the Taylor series of Eq. taylor (eps = 0)."""
    Xt, ZA, Ys, ms, ZB = _two_clusters(seed)
    R = ZA - ZB
    _, D1, D2, D3, D4 = _D_tensors(R)
    y = Ys - ZB
    M = ms.sum()
    Q = np.einsum("b,bi,bj->ij", ms, y, y)
    H = -np.einsum("b,bi,bj,bk->ijk", ms, y, y, y)
    acc, _ = oracle.cluster_far(Xt, ZA, Ys, ms, ZB, 4, 0.0, "standard")
    for a in range(len(Xt)):
        x = Xt[a] - ZA
        ref = (-M * D1 - M * D2 @ x
               - 0.5 * np.einsum("ijk,jk->i", D3, Q + M * np.outer(x, x))
               - (1.0 / 6.0) * np.einsum("ijkl,jkl->i", D4,
                                         H + 3.0 * np.einsum("jk,l->jkl", Q, x)
                                         + M * np.einsum("j,k,l->jkl", x, x, x)))
        np.testing.assert_allclose(acc[a], ref, rtol=1e-12, atol=1e-14 * np.linalg.norm(ref))


def test_p4_potential_matches_eq_potential():
    Xt, ZA, Ys, ms, ZB = _two_clusters(4)
    R = ZA - ZB
    D0, D1, D2, D3, D4 = _D_tensors(R)
    y = Ys - ZB
    M = ms.sum()
    Q = np.einsum("b,bi,bj->ij", ms, y, y)
    H = -np.einsum("b,bi,bj,bk->ijk", ms, y, y, y)
    X4 = np.einsum("b,bi,bj,bk,bl->ijkl", ms, y, y, y, y)
    _, pot = oracle.cluster_far(Xt, ZA, Ys, ms, ZB, 4, 0.0, "standard")
    for a in range(len(Xt)):
        x = Xt[a] - ZA
        xx = np.outer(x, x)
        ref = (M * D0 + D1 @ x * M + 0.5 * np.einsum("ij,ij", D2, Q + M * xx)
               + (1 / 6) * np.einsum("ijk,ijk", D3, H + 3 * np.einsum("ij,k->ijk", Q, x)
                                     + M * np.einsum("i,j,k->ijk", x, x, x))
               + (1 / 24) * np.einsum("ijkl,ijkl", D4, X4 + 4 * np.einsum("ijk,l->ijkl", H, x)
                                      + 6 * np.einsum("ij,k,l->ijkl", Q, x, x)
                                      + M * np.einsum("i,j,k,l->ijkl", x, x, x, x)))
        assert abs(pot[a] - ref) <= 1e-12 * abs(ref)


def test_traceless_moments_of_eq_quad_mom_give_three_times_raw():
    """Eqs. quad_mom / octo_mom against D tensors: the printed traceless
    moments contract with the (traceless) D tensors to 3x / -15x the raw
    moments used by the oracle (eps = 0)."""
    Xt, ZA, Ys, ms, ZB = _two_clusters(5)
    _, _, D2, D3, _ = _D_tensors(ZA - ZB)
    y = Ys - ZB
    q2 = (y * y).sum(1)
    I = np.eye(3)
    Qtl = np.einsum("b,bij->ij", ms, 3 * np.einsum("bi,bj->bij", y, y) - q2[:, None, None] * I)
    Qraw = np.einsum("b,bi,bj->ij", ms, y, y)
    assert abs(np.einsum("ij,ij", D2, Qtl) - 3 * np.einsum("ij,ij", D2, Qraw)) < 1e-12 * abs(np.einsum("ij,ij", D2, Qtl))
    Htl = np.einsum("b,bijk->ijk", ms, 15 * np.einsum("bi,bj,bk->bijk", y, y, y)
                    - 3 * q2[:, None, None, None] * (np.einsum("ij,bk->bijk", I, y)
                                                     + np.einsum("jk,bi->bijk", I, y)
                                                     + np.einsum("ik,bj->bijk", I, y)))
    Hraw = np.einsum("b,bi,bj,bk->ijk", ms, y, y, y)
    lhs = np.einsum("ijk,ijk", D3, Htl)
    assert abs(lhs - 15 * np.einsum("ijk,ijk", D3, Hraw)) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_p2_conserving_matches_eq_aaB1(seed):
    """Eq. aaB1, read with D^k := R^-k, <u,v>_D := R D_ij u^i v^j (D_ij of Eq. Dij),
    xi = x_a / R, Q = sum m y y about the COM of B, M_b -> M_B (eps = 0)."""
    Xt, ZA, Ys, ms, ZB = _two_clusters(seed)
    R = ZA - ZB
    r = np.linalg.norm(R)
    nR = R / r
    _, _, D2, _, _ = _D_tensors(R)
    y = Ys - ZB
    M = ms.sum()
    Q = np.einsum("b,bi,bj->ij", ms, y, y)
    acc, _ = oracle.cluster_far(Xt, ZA, Ys, ms, ZB, 2, 0.0, "conserving")

    def dprod(u, v):  # <u, v>_D with v a vector or a matrix (contracting its first index)
        return r * np.einsum("ij,i,j...->...", D2, u, v)

    for a in range(len(Xt)):
        xi = (Xt[a] - ZA) / r
        ref = (-M * (r ** -2 * (1.0 - xi @ nR) + dprod(xi, nR)) * (nR + xi)
               - dprod(nR, Q) * r ** -2 + (nR @ Q) * r ** -4)
        np.testing.assert_allclose(acc[a], ref, rtol=1e-12, atol=1e-14 * np.linalg.norm(ref))


def test_p1_conserving_is_pointed_at_source_com():
    """Zeroth-order (p=1) conserving force: -M_B (X_a - Z_B)(R^2+eps^2)^(-3/2)."""
    Xt, ZA, Ys, ms, ZB = _two_clusters(6)
    eps = 0.05
    R = ZA - ZB
    acc, _ = oracle.cluster_far(Xt, ZA, Ys, ms, ZB, 1, eps, "conserving")
    ref = -ms.sum() * (Xt - ZB) * (R @ R + eps * eps) ** -1.5
    np.testing.assert_allclose(acc, ref, rtol=1e-13)


def test_p1_standard_is_constant_acceleration():
    """Sec. 3.1: zeroth-order FMM gives every particle of A the same acceleration."""
    Xt, ZA, Ys, ms, ZB = _two_clusters(7)
    acc, _ = oracle.cluster_far(Xt, ZA, Ys, ms, ZB, 1, 0.0, "standard")
    R = ZA - ZB
    ref = -ms.sum() * R / np.linalg.norm(R) ** 3
    np.testing.assert_allclose(acc, np.tile(ref, (len(Xt), 1)), rtol=1e-13)


# ---------------------------------------------------------------------------
# Direct sum and tree-based forces.
# ---------------------------------------------------------------------------
def test_direct_matches_numpy_broadcast():
    pos, m = uniform_ball(300, 11)
    eps = 0.01
    d = pos[:, None, :] - pos[None, :, :]
    r2 = (d * d).sum(-1) + eps * eps
    np.fill_diagonal(r2, np.inf)
    ref = -(m[:, None, None] * m[None, :, None] * d * r2[..., None] ** -1.5).sum(1)
    np.testing.assert_allclose(oracle.direct(pos, m, eps), ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("p", [1, 4])
@pytest.mark.parametrize("variant", ["standard", "conserving"])
def test_theta_zero_reproduces_direct_sum(p, variant):
    """theta -> 0: only exact pairs and single-particle nodes remain (Eq. jia)."""
    pos, m = uniform_ball(700, 12)
    ref = oracle.direct(pos, m, 1e-3)
    t = oracle.Tree(pos, m, n_leaf=8, theta=0.0)
    f = t.forces(p, 1e-3, variant)
    err = np.linalg.norm(f - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() < 1e-13


@pytest.fixture(scope="module")
def ball2k():
    pos, m = uniform_ball(2048, 210707166)
    return pos, m, oracle.direct(pos, m, 1e-3)


def _erms(f, ref):
    return float(np.sqrt(np.mean(((f - ref) ** 2).sum(1) / (ref ** 2).sum(1))))


def test_error_falls_with_order_and_angle(ball2k):
    pos, m, ref = ball2k
    for variant in ("standard", "conserving"):
        errs = {}
        for theta in (0.2, 0.4, 0.6, 0.8):
            t = oracle.Tree(pos, m, n_leaf=16, theta=theta)
            for p in (1, 2, 4, 6):
                errs[theta, p] = _erms(t.forces(p, 1e-3, variant), ref)
        for theta in (0.2, 0.4, 0.6, 0.8):
            e = [errs[theta, p] for p in (1, 2, 4, 6)]
            assert all(e[i + 1] < e[i] for i in range(3)), (variant, theta, e)
        for p in (1, 2, 4, 6):
            e = [errs[th, p] for th in (0.2, 0.4, 0.6, 0.8)]
            assert all(e[i] < e[i + 1] for i in range(3)), (variant, p, e)


def test_realignment_keeps_the_accuracy_order(ball2k):
    """On a tree workload the realigned force keeps the standard force's order
    of accuracy but not its constant: the conserving/standard error ratio at
    fixed p stays bounded (measured 2.8-5.6 here for p = 1..6).  The paper's
    statement that accuracy is not affected (Sec. 4) is about its two-body
    distance test, where the ratio is 0.7-1.1 (pinned in
    test_oracle_outputs.py).  Its top-order term is a Taylor term of
    g = |r|^-3, which is not harmonic, so its sum over a source cell lacks the
    cancellation of the harmonic standard remainder."""
    pos, m, ref = ball2k
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.5)
    for p in (2, 4, 6):
        es = _erms(t.forces(p, 1e-3, "standard"), ref)
        ec = _erms(t.forces(p, 1e-3, "conserving"), ref)
        assert ec / es < 6.0, (p, es, ec)


@pytest.mark.parametrize("p", [1, 2, 4, 6])
def test_momentum_balance_and_torque(ball2k, p):
    """Eq. netforce: zero net force in both variants.  Eq. total_torque: the
    standard expansion leaves a net torque for p >= 2 (none at p = 1, Sec. 3.1);
    the realigned forces have none (Sec. 3.2)."""
    pos, m, _ = ball2k
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.6)
    ds = oracle.diagnostics(pos, m, t.forces(p, 1e-3, "standard"))
    dc = oracle.diagnostics(pos, m, t.forces(p, 1e-3, "conserving"))
    assert ds[18] < 1e-14 and dc[18] < 1e-14
    assert dc[19] < 1e-14
    if p == 1:
        assert ds[19] < 1e-14
    else:
        assert ds[19] > 1e-9


def test_forces_independent_of_thread_count(ball2k):
    pos, m, _ = ball2k
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.5)
    old = oracle.set_threads(0)
    try:
        oracle.set_threads(1)
        f1 = t.forces(4, 1e-3, "conserving")
        oracle.set_threads(4)
        f4 = t.forces(4, 1e-3, "conserving")
    finally:
        oracle.set_threads(old)
    assert np.array_equal(f1, f4)


def test_forces_on_subset_equal_full_evaluation(ball2k):
    pos, m, _ = ball2k
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.5)
    full = t.forces(4, 1e-3, "standard")
    idx = np.array([5, 17, 1999, 0, 1024])
    assert np.array_equal(t.forces(4, 1e-3, "standard", targets=idx), full[idx])


def test_input_permutation_leaves_forces_unchanged():
    pos, m = plummer(1500, 13)
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.6)
    f = t.forces(4, 1e-3, "conserving")
    perm = _rng(3).permutation(len(m))
    t2 = oracle.Tree(pos[perm], m[perm], n_leaf=16, theta=0.6)
    f2 = t2.forces(4, 1e-3, "conserving")
    np.testing.assert_allclose(f2, f[perm], rtol=1e-13, atol=1e-15 * np.abs(f).max())


def test_p2_standard_torque_matches_closed_form():
    """Eq. total_torque at p = 2.  Two clusters in opposite octants of the
    root cube are joined by a single far pair; the near forces inside each
    cluster are exact central pair forces (no torque), and the truncated far
    forces a_a = -M_B grad phi(R) - M_B Phi x_a (x_a about Z_A, Phi the second
    derivatives of the softened kernel at R = Z_A - Z_B) leave the net torque
    tau_i = -eps_ijk Phi_kl (M_B Q_A + M_A Q_B)_jl, with Q the raw second
    moments about each cluster's centre of mass."""
    rng = _rng(21)
    A = rng.normal(size=(30, 3)) * 0.15 + np.array([-1.0, -1.0, -1.0])
    B = rng.normal(size=(40, 3)) * 0.2 + np.array([1.0, 0.8, 1.1])
    pos = np.vstack([A, B])
    m = rng.uniform(0.5, 1.5, len(pos))
    eps = 0.05
    t = oracle.Tree(pos, m, n_leaf=64, theta=0.5)
    far, near = t.lists()
    assert len(far) == 1 and len(near) == 2
    F = t.forces(2, eps, "standard")
    tau = np.cross(pos, F).sum(0)
    mA, mB = m[:30], m[30:]
    MA, MB = mA.sum(), mB.sum()
    ZA = (mA[:, None] * A).sum(0) / MA
    ZB = (mB[:, None] * B).sum(0) / MB
    QA = np.einsum("a,ai,aj->ij", mA, A - ZA, A - ZA)
    QB = np.einsum("a,ai,aj->ij", mB, B - ZB, B - ZB)
    R = ZA - ZB
    s = R @ R + eps * eps
    Phi = np.eye(3) * s ** -1.5 - 3.0 * np.outer(R, R) * s ** -2.5
    lc = np.zeros((3, 3, 3))
    lc[0, 1, 2] = lc[1, 2, 0] = lc[2, 0, 1] = 1.0
    lc[0, 2, 1] = lc[2, 1, 0] = lc[1, 0, 2] = -1.0
    closed = -np.einsum("ijk,kl,jl->i", lc, Phi, MB * QA + MA * QB)
    assert np.linalg.norm(closed) > 1e-4
    assert np.linalg.norm(tau - closed) <= 1e-9 * np.linalg.norm(closed)
    # the realigned forces of the same tree carry no torque
    tc = np.cross(pos, t.forces(2, eps, "conserving")).sum(0)
    assert np.linalg.norm(tc) <= 1e-12 * np.linalg.norm(closed)
