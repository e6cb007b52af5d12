"""Pins of the conserving variant with the projection scalar kept to a degree
K above the default p-1 (Sec. 3.2: the expansion of the scalar of Eq.
abnab-expansion may keep more terms than the first order).

Definition: the standard order-p pair force a (gradient of the truncated Eq.
taylor) is projected onto u = X_a - Y_b (Eq. realign), a' = ((a.u)/|u|^2) u,
and the scalar is replaced by its Taylor polynomial of degree K in
delta = x_a - y_b.

Pins: sympy's series of that scalar (the defining expression, expanded
symbolically); an identity derived by hand and evaluated here with scipy's
Gegenbauer polynomials and numpy polynomial division; the default K = p-1;
central and antisymmetric pair forces (no net force, no net torque).
"""

import math

import numpy as np
import pytest
import scipy.special as sps
import sympy as sp

import oracle
from paper_2107_07166_amd.generators import uniform_ball


def _sympy_scalar_force(R, dnum, eps, p, K):
    t = sp.Symbol("t")
    dx, dy, dz = sp.symbols("dx dy dz")
    Rs = [sp.Float(v, 30) for v in R]
    e2 = sp.Float(eps, 30) ** 2
    phi = -((Rs[0] + t * dx) ** 2 + (Rs[1] + t * dy) ** 2 + (Rs[2] + t * dz) ** 2 + e2) ** sp.Rational(-1, 2)
    Tp = sp.series(phi, t, 0, p + 1).removeO().subs(t, 1)
    grad = [sp.diff(Tp, v) for v in (dx, dy, dz)]
    tsub = {dx: t * dnum[0], dy: t * dnum[1], dz: t * dnum[2]}
    a_t = [-g.subs(tsub) for g in grad]
    u_t = [Rs[k] + t * dnum[k] for k in range(3)]
    scal = (a_t[0] * u_t[0] + a_t[1] * u_t[1] + a_t[2] * u_t[2]) / (u_t[0] ** 2 + u_t[1] ** 2 + u_t[2] ** 2)
    sK = float(sp.series(scal, t, 0, K + 1).removeO().subs(t, 1))
    return sK * (np.array(R) + np.array(dnum))


@pytest.mark.parametrize("p,K", [(1, 1), (1, 3), (2, 2), (2, 3), (3, 4), (4, 5), (4, 6), (5, 6)])
def test_scalar_degree_matches_sympy_series(p, K):
    rng = np.random.default_rng(50 + 10 * p + K)
    for trial in range(3):
        R = rng.normal(size=3)
        R *= rng.uniform(1.0, 3.0) / np.linalg.norm(R)
        x = rng.normal(size=3) * 0.25
        y = rng.normal(size=3) * 0.25
        eps = [0.0, 1e-3, 0.2][trial]
        ref = _sympy_scalar_force(R, x - y, eps, p, K)
        acc, _ = oracle.pair_far(R, x, y, 1.0, p, eps, "conserving", scalar_degree=K)
        np.testing.assert_allclose(acc, ref, rtol=1e-11, atol=1e-13 * np.linalg.norm(ref))


def _identity_force(R, d, eps, p, K):
    """The same force through a hand-derived identity: with G_n the degree-n
    part of g(R + delta), g = (|r|^2 + eps^2)^(-3/2), the projected standard
    scalar is -T_{p-1}[g] + G_{p-1}(delta) (u.delta)/|u|^2, whose second factor
    starts at degree 1; so the degree-K scalar is -T_{p-1}[g] + G_{p-1} times
    the Taylor polynomial of (u.delta)/|u|^2 of degree K-p+1.  G_n from the
    Gegenbauer generating function, the rational function's series by
    polynomial long division."""
    c0 = R @ R + eps * eps
    c1 = 2.0 * (R @ d)
    c2 = d @ d
    h = math.sqrt(c2 / c0)
    x = -c1 / (2.0 * math.sqrt(c0 * c2))
    G = [c0 ** -1.5 * sps.eval_gegenbauer(n, 1.5, x) * h ** n for n in range(p)]
    # (u.delta)/|u|^2 along t: numerator t (R.d) + t^2 (d.d), denominator
    # R.R + 2 t R.d + t^2 d.d (no softening in the projection)
    num = [0.0, R @ d, d @ d]
    den = [R @ R, 2.0 * (R @ d), d @ d]
    m = K - p + 1
    w = np.zeros(m + 1)
    rem = list(num) + [0.0] * (m + 3)
    for n in range(m + 1):
        w[n] = rem[n] / den[0]
        for j in range(3):
            rem[n + j] -= w[n] * den[j]
    scal = -sum(G) + G[p - 1] * w.sum()
    return scal * (R + d)


@pytest.mark.parametrize("p,K", [(1, 2), (2, 4), (3, 3), (4, 5), (4, 6), (6, 7), (7, 9)])
def test_scalar_degree_matches_derived_identity(p, K):
    rng = np.random.default_rng(90 + 10 * p + K)
    for _ in range(20):
        R = rng.normal(size=3)
        R *= rng.uniform(1.0, 3.0) / np.linalg.norm(R)
        x = rng.normal(size=3) * 0.3
        y = rng.normal(size=3) * 0.3
        eps = rng.choice([0.0, 1e-3, 0.1])
        ref = _identity_force(R, x - y, eps, p, K)
        acc, _ = oracle.pair_far(R, x, y, 1.0, p, eps, "conserving", scalar_degree=K)
        np.testing.assert_allclose(acc, ref, rtol=1e-12, atol=1e-14 * np.linalg.norm(ref))


@pytest.mark.parametrize("p", [1, 2, 4, 7])
def test_default_degree_is_p_minus_one(p):
    rng = np.random.default_rng(7 + p)
    R = np.array([1.2, -0.7, 0.4])
    x, y = rng.normal(size=3) * 0.2, rng.normal(size=3) * 0.2
    a0, _ = oracle.pair_far(R, x, y, 0.7, p, 1e-3, "conserving")
    a1, _ = oracle.pair_far(R, x, y, 0.7, p, 1e-3, "conserving", scalar_degree=max(p - 1, 0))
    np.testing.assert_allclose(a1, a0, rtol=1e-14)


def test_scalar_degree_rejected_where_undefined():
    R, x, y = np.array([2.0, 0.0, 0.0]), np.zeros(3), np.full(3, 0.1)
    for variant, p, K in (("standard", 3, 4), ("conserving", 4, 2), ("conserving", 4, 13),
                          ("conserving_r2", 1, 2)):
        with pytest.raises(ValueError):
            oracle.pair_far(R, x, y, 1.0, p, 1e-3, variant, scalar_degree=K)


@pytest.mark.parametrize("p", [2, 4])
def test_scalar_degree_tree_forces_conserve_momenta_and_gain_accuracy(p):
    """Each realigned pair force is central and antisymmetric, so the tree
    sums have no net force (Eq. netforce) and no net torque (Eq. total_torque)
    at every K; and keeping more terms of the scalar brings the force closer
    to the direct sum (Sec. 3.2: more terms for better accuracy)."""
    pos, m = uniform_ball(1200, 61)
    ref = oracle.direct(pos, m, 1e-3)
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.5)
    errs = []
    for K in (p - 1, p, p + 1):
        f = t.forces(p, 1e-3, "conserving", scalar_degree=K)
        d = oracle.diagnostics(pos, m, f)
        assert d[18] < 1e-14 and d[19] < 1e-14, K
        errs.append(float(np.sqrt(np.mean(((f - ref) ** 2).sum(1) / (ref ** 2).sum(1)))))
    assert errs[0] > errs[1] > errs[2], errs


def test_scalar_degree_zero_theta_is_direct():
    pos, m = uniform_ball(500, 62)
    ref = oracle.direct(pos, m, 1e-3)
    f = oracle.Tree(pos, m, n_leaf=8, theta=0.0).forces(3, 1e-3, "conserving", scalar_degree=5)
    np.testing.assert_allclose(f, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
