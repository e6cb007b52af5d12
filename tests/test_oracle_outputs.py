"""Pins of the oracle's remaining outputs: the momentum diagnostics (all 20
slots), the direct and tree-level potentials, and the tree assembly of the
far field for one accepted node pair.

Paper: Korobkin et al., arXiv:2107.07166.  Eq. netforce (net force), Eq.
total_torque (net torque), Eq. jia (softened pair potential), Eq. taylor
(truncated far-field potential).  Every reference here is computed with
numpy from the definitions, with math.fsum for the sums, not by the oracle's
own routines.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2107_07166_amd.generators import irregular_pair, plummer, uniform_ball


def _fsum3(v):
    return np.array([math.fsum(v[:, k]) for k in range(3)])


def _diag_numpy(pos, m, F, v):
    """The 20 diagnostics slots from their definitions (torque and angular
    momentum about the mass-weighted centre)."""
    M = math.fsum(m)
    cm = _fsum3(m[:, None] * pos) / M
    r = pos - cm
    out = np.zeros(20)
    out[0:3] = _fsum3(F)
    fn = np.sqrt((F * F).sum(1))
    rn = np.sqrt((r * r).sum(1))
    out[3] = math.fsum(fn)
    out[4:7] = _fsum3(np.cross(r, F))
    out[7] = math.fsum(rn * fn)
    out[8:11] = _fsum3(m[:, None] * v)
    out[11:14] = _fsum3(m[:, None] * np.cross(r, v))
    out[14] = M
    out[15:18] = cm
    out[18] = np.linalg.norm(out[0:3]) / out[3]
    out[19] = np.linalg.norm(out[4:7]) / out[7]
    return out


def test_diagnostics_all_slots_match_numpy():
    """Eqs. netforce and total_torque: sum F, sum |F|, sum (X-Xcm) x F,
    sum |X-Xcm||F|, P, L, total mass, centre of mass, and the two relative
    residuals, on inputs with a displaced centre of mass and non-zero momenta."""
    rng = np.random.default_rng(101)
    n = 1500
    pos = rng.normal(size=(n, 3)) * np.array([1.0, 0.5, 2.0]) + np.array([3.0, -1.0, 0.5])
    m = rng.uniform(0.2, 2.0, n)
    F = rng.normal(size=(n, 3)) + np.array([0.1, -0.2, 0.05])
    v = rng.normal(size=(n, 3)) + np.array([0.0, 0.3, -0.1])
    got = oracle.diagnostics(pos, m, F, vel=v)
    ref = _diag_numpy(pos, m, F, v)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)


def test_diagnostics_without_velocities_zero_momenta():
    rng = np.random.default_rng(102)
    pos = rng.normal(size=(300, 3))
    m = rng.uniform(0.5, 1.5, 300)
    F = rng.normal(size=(300, 3))
    got = oracle.diagnostics(pos, m, F)
    ref = _diag_numpy(pos, m, F, np.zeros_like(pos))
    assert np.all(got[8:14] == 0.0)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)


def test_diagnostics_central_pair_forces_have_no_net_force_or_torque():
    """Forces made of equal and opposite central pair terms (Eq. netforce,
    Eq. total_torque with central pairs): both relative residuals vanish to
    rounding, whatever the origin of the coordinates."""
    rng = np.random.default_rng(103)
    n = 200
    pos = rng.normal(size=(n, 3)) + 5.0
    m = rng.uniform(0.5, 1.5, n)
    F = np.zeros((n, 3))
    for _ in range(2000):
        a, b = rng.choice(n, 2, replace=False)
        f = rng.normal() * (pos[a] - pos[b])
        F[a] += f
        F[b] -= f
    d = oracle.diagnostics(pos, m, F)
    assert d[18] < 1e-14 and d[19] < 1e-14
    # a uniform extra force is a pure net force; a tangential pair a pure torque
    d2 = oracle.diagnostics(pos, m, F + np.array([0.0, 0.0, 1e-3]))
    assert d2[18] > 1e-6


def test_direct_potential_matches_numpy_broadcast():
    """Eq. jia with Plummer softening: phi_a = -G sum_{b != a} m_b (r^2 + eps^2)^(-1/2)."""
    pos, m = uniform_ball(400, 17)
    eps, G = 0.02, 1.7
    d = pos[:, None, :] - pos[None, :, :]
    r2 = (d * d).sum(-1) + eps * eps
    np.fill_diagonal(r2, np.inf)
    ref = -G * (m[None, :] / np.sqrt(r2)).sum(1)
    _, pot = oracle.direct(pos, m, eps, G=G, with_potential=True)
    np.testing.assert_allclose(pot, ref, rtol=1e-13)


def test_direct_skips_coincident_unsoftened_pairs():
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    m = np.array([1.0, 2.0, 3.0])
    f, pot = oracle.direct(pos, m, 0.0, with_potential=True)
    np.testing.assert_allclose(f[0], [3.0, 0.0, 0.0], rtol=1e-15)
    np.testing.assert_allclose(pot, [-3.0, -3.0, -3.0], rtol=1e-15)
    np.testing.assert_allclose(f[1], [6.0, 0.0, 0.0], rtol=1e-15)
    np.testing.assert_allclose(f[2], [-9.0, 0.0, 0.0], rtol=1e-15)


@pytest.mark.parametrize("p", [1, 3, 6])
@pytest.mark.parametrize("variant", ["standard", "conserving"])
def test_theta_zero_tree_potential_equals_direct(p, variant):
    """theta = 0 accepts no pair of multi-particle nodes, so the tree-level
    potential is the exact softened sum of Eq. jia for every order."""
    pos, m = plummer(900, 33)
    f_ref, pot_ref = oracle.direct(pos, m, 1e-3, with_potential=True)
    t = oracle.Tree(pos, m, n_leaf=8, theta=0.0)
    f, pot = t.forces(p, 1e-3, variant, with_potential=True)
    np.testing.assert_allclose(pot, pot_ref, rtol=1e-13)
    np.testing.assert_allclose(f, f_ref, rtol=1e-12, atol=1e-13 * np.abs(f_ref).max())


def test_potential_error_falls_with_order():
    pos, m = uniform_ball(1500, 34)
    _, ref = oracle.direct(pos, m, 1e-3, with_potential=True)
    t = oracle.Tree(pos, m, n_leaf=16, theta=0.6)
    errs = []
    for p in (1, 2, 4, 6):
        _, pot = t.forces(p, 1e-3, "standard", with_potential=True)
        errs.append(float(np.sqrt(np.mean((pot - ref) ** 2) / np.mean(ref ** 2))))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs


def test_tree_assembly_for_one_far_pair_at_order_two():
    """Two clusters in opposite octants joined by one accepted node pair: the
    tree-level force and potential of every particle equal the exact softened
    sum over its own cluster plus, over the other cluster, the second-order
    Taylor expansion of Eq. taylor about the two centres of mass,
    m_b (phi(R) + grad phi(R).delta + delta.Phi(R).delta / 2) and its
    negative gradient in delta (G = 1.3 scales both)."""
    rng = np.random.default_rng(35)
    A = rng.normal(size=(25, 3)) * 0.15 + np.array([-1.0, -1.0, -1.0])
    B = rng.normal(size=(35, 3)) * 0.2 + np.array([1.0, 0.9, 1.1])
    pos = np.vstack([A, B])
    m = rng.uniform(0.5, 1.5, len(pos))
    eps, G = 0.05, 1.3
    t = oracle.Tree(pos, m, n_leaf=36, theta=0.5)
    far, near = t.lists()
    assert len(far) == 1 and len(near) == 2
    f, pot = t.forces(2, eps, "standard", G=G, with_potential=True)

    def phi_parts(R):
        s = R @ R + eps * eps
        return -s ** -0.5, R * s ** -1.5, np.eye(3) * s ** -1.5 - 3.0 * np.outer(R, R) * s ** -2.5

    groups = [(np.arange(25), np.arange(25, 60)), (np.arange(25, 60), np.arange(25))]
    for own, other in groups:
        Z_own = (m[own, None] * pos[own]).sum(0) / m[own].sum()
        Z_oth = (m[other, None] * pos[other]).sum(0) / m[other].sum()
        R = Z_own - Z_oth
        p0, p1, p2 = phi_parts(R)
        for a in own:
            acc = np.zeros(3)
            ph = []
            for b in own:
                if b == a:
                    continue
                d = pos[a] - pos[b]
                s = d @ d + eps * eps
                acc -= m[b] * d * s ** -1.5
                ph.append(-m[b] * s ** -0.5)
            for b in other:
                dl = (pos[a] - Z_own) - (pos[b] - Z_oth)
                acc -= m[b] * (p1 + p2 @ dl)
                ph.append(m[b] * (p0 + p1 @ dl + 0.5 * dl @ p2 @ dl))
            np.testing.assert_allclose(f[a], G * m[a] * acc, rtol=1e-12, atol=1e-14 * np.abs(f).max())
            assert abs(pot[a] - G * math.fsum(ph)) <= 1e-12 * abs(pot[a])


# ---------------------------------------------------------------------------
# Accuracy of the realigned force (Sec. 4: accuracy not affected by the
# realignment in the two-body test of the distance figure).
# ---------------------------------------------------------------------------
def _erms(f, ref):
    return float(np.sqrt(np.mean(((f - ref) ** 2).sum(1) / (ref ** 2).sum(1))))


@pytest.mark.parametrize("sep", [3.6, 8.0])
def test_realignment_keeps_accuracy_in_the_two_body_setup(sep):
    """The setup of the paper's distance test: two irregular bodies, each one
    leaf, joined by one accepted pair (eps = 0).  The realigned force's error
    against the direct sum stays within 1.5x of the standard one at every
    order (measured 0.67-1.09)."""
    pos, m = irregular_pair(800, 5, sep)
    ref = oracle.direct(pos, m, 0.0)
    t = oracle.Tree(pos, m, n_leaf=800, theta=0.99)
    assert t.n_m2l == 1
    for p in (1, 2, 3, 4, 5, 6):
        es = _erms(t.forces(p, 0.0, "standard"), ref)
        ec = _erms(t.forces(p, 0.0, "conserving"), ref)
        assert ec <= 1.5 * es, (p, es, ec)
