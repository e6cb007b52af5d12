"""Pins of the oracle's realigned-by-magnitude zeroth-order far field
(variant "conserving_r2": Eq. realign2 with n_ab expanded as in Eq.
nab-expansion; summed over a source node it is Eq. aaB0)."""
import numpy as np
import pytest

import oracle
from paper_2107_07166_amd.generators import uniform_ball


def _two_clusters(seed, nb=40, na=7, dist=3.0, size=0.3):
    rng = np.random.default_rng(seed)
    Ys = rng.normal(size=(nb, 3)) * size
    ms = rng.uniform(0.5, 1.5, nb)
    ZB = (ms[:, None] * Ys).sum(0) / ms.sum()
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    Xt = rng.normal(size=(na, 3)) * size + dist * direction
    ZA = Xt.mean(0)
    return Xt, ZA, Ys, ms, ZB


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cluster_sum_matches_eq_aaB0(seed):
    """Eq. aaB0 (eps = 0, G = 1): -(M_B/R^2) [n_R + x_perp/R - (x.n_R) x/R^2
    - n_R.Q_B/(M_B R^2)] with Q_B the raw second moment of B about its COM
    and x the target's offset from the expansion centre of A."""
    Xt, ZA, Ys, ms, ZB = _two_clusters(seed)
    R = ZA - ZB
    r = np.linalg.norm(R)
    n = R / r
    y = Ys - ZB
    M = ms.sum()
    Q = np.einsum("b,bi,bj->ij", ms, y, y)
    acc, _ = oracle.cluster_far(Xt, ZA, Ys, ms, ZB, 1, 0.0, "conserving_r2")
    for a in range(len(Xt)):
        x = Xt[a] - ZA
        xperp = x - n * (n @ x)
        ref = -(M / r ** 2) * (n + xperp / r - (x @ n) * x / r ** 2 - (n @ Q) / (M * r ** 2))
        np.testing.assert_allclose(acc[a], ref, rtol=1e-12, atol=1e-15 * np.linalg.norm(ref))


def test_pair_is_central_and_antisymmetric():
    """Each pair force lies on X_a - Y_b (no pair torque) and obeys action =
    reaction (R -> -R, x <-> y)."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        R = rng.normal(size=3) * 3.0
        x, y = rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.3
        ma, mb, eps = 0.7, 1.3, 0.05
        ab, _ = oracle.pair_far(R, x, y, mb, 1, eps, "conserving_r2")
        ba, _ = oracle.pair_far(-R, y, x, ma, 1, eps, "conserving_r2")
        u = R + x - y
        assert np.linalg.norm(np.cross(ab, u)) <= 1e-14 * np.linalg.norm(ab) * np.linalg.norm(u)
        np.testing.assert_allclose(ma * ab, -mb * ba, rtol=1e-14, atol=1e-16)


def test_second_order_in_delta_against_exact_realignment():
    """Eq. realign2 itself, -|a0| n_ab with |a0| = |R| (R^2+eps^2)^(-3/2) and the
    exact unit vector: the expansion of n_ab to first order leaves an error
    that falls as (|delta|/|R|)^2."""
    R = np.array([2.0, -1.0, 1.5])
    eps = 0.02
    rng = np.random.default_rng(5)
    d0 = rng.normal(size=3) * 0.2
    errs = []
    for s in (1.0, 0.5, 0.25, 0.125):
        x, y = s * d0, np.zeros(3)
        acc, _ = oracle.pair_far(R, x, y, 1.0, 1, eps, "conserving_r2")
        u = R + x - y
        r = np.linalg.norm(R)
        exact = -r * (r * r + eps * eps) ** -1.5 * u / np.linalg.norm(u)
        errs.append(np.linalg.norm(acc - exact) / np.linalg.norm(exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.5 < q < 4.5 for q in ratios), (errs, ratios)


@pytest.fixture(scope="module")
def ball2k():
    pos, m = uniform_ball(2048, 210707166)
    return pos, m, oracle.direct(pos, m, 1e-3)


def test_tree_forces_keep_momentum_and_angular_momentum(ball2k):
    """Sec. 3.2: with every far-field pair force central and antisymmetric the
    net force and the net torque vanish (to rounding)."""
    pos, m, _ = ball2k
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.6)
    d = oracle.diagnostics(pos, m, t.forces(1, 1e-3, "conserving_r2"))
    assert d[18] < 1e-14 and d[19] < 1e-14


def test_theta_zero_reproduces_direct_sum():
    pos, m = uniform_ball(700, 12)
    ref = oracle.direct(pos, m, 1e-3)
    t = oracle.Tree(pos, m, n_leaf=8, theta=0.0)
    f = t.forces(1, 1e-3, "conserving_r2")
    err = np.linalg.norm(f - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() < 1e-13


def test_error_two_thirds_of_projected_zeroth_order(ball2k):
    """Both zeroth-order realignments point each pair force exactly along
    X_a - Y_b to first order; they differ in the magnitude.  Projection
    (Eq. realign at p = 1) gives |R + delta| g(R), a relative error of
    3 n_R.delta/|R| against 1/|R + delta|^2; Eq. realign2 gives
    (1 - n_R.delta/|R|) |n_R + delta/|R|| / |R|^2, an error of
    2 n_R.delta/|R|.  The tree errors against the direct sum keep that ratio."""
    pos, m, ref = ball2k
    cases = [(pos, m, ref)]
    from paper_2107_07166_amd.generators import plummer
    pp, pm = plummer(2048, 3)
    cases.append((pp, pm, oracle.direct(pp, pm, 1e-3)))

    def erms(f, r):
        return float(np.sqrt(np.mean(((f - r) ** 2).sum(1) / (r ** 2).sum(1))))

    for p_, m_, r_ in cases:
        last = None
        for theta in (0.3, 0.5, 0.7):
            t = oracle.Tree(p_, m_, n_leaf=16, theta=theta)
            er = erms(t.forces(1, 1e-3, "conserving_r2"), r_)
            ec = erms(t.forces(1, 1e-3, "conserving"), r_)
            assert 0.5 < er / ec < 0.85, (theta, er, ec)
            assert last is None or er > last
            last = er


def test_only_zeroth_order_is_accepted(ball2k):
    pos, m, _ = ball2k
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.5)
    with pytest.raises(Exception):
        t.forces(2, 1e-3, "conserving_r2")
