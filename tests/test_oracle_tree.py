"""Pins of the oracle's tree, keys and walk.

The paper does not describe tree construction (it only uses "tree nodes",
their centres of mass and the r_max of Eq. mac_criterion); the readings
implemented by the oracle are checked here against brute force and against
the invariants any valid mutual FMM walk must satisfy: every unordered
particle pair is covered exactly once, accepted pairs satisfy Eq.
mac_criterion, rejected pairs of leaves do not.
"""

import numpy as np
import pytest

import oracle
from paper_2107_07166_amd.generators import plummer, uniform_ball


def _brute_keys(pos):
    lo = pos.min(0)
    ext = (pos.max(0) - lo).max()
    if ext == 0.0:
        ext = 1.0
    scale = 2097152.0 / ext
    keys = []
    for p in pos:
        q = [min(2 ** 21 - 1, int(np.floor((p[d] - lo[d]) * scale))) for d in range(3)]
        k = 0
        for i in range(21):
            k |= ((q[0] >> i) & 1) << (3 * i + 2)
            k |= ((q[1] >> i) & 1) << (3 * i + 1)
            k |= ((q[2] >> i) & 1) << (3 * i)
        keys.append(k)
    return np.array(keys, dtype=np.uint64), lo, ext, scale


def test_keys_and_order_match_bruteforce():
    pos, m = plummer(400, 5)
    t = oracle.Tree(pos, m, n_leaf=8, theta=0.5)
    keys, order = t.keys()
    ref, lo, ext, scale = _brute_keys(pos)
    assert np.array_equal(keys, ref)
    bb = t.bbox()
    assert np.array_equal(bb[:3], lo) and bb[3] == ext and bb[4] == scale
    assert np.array_equal(order, np.argsort(ref, kind="stable"))


def _check_nodes(t, pos, m, n_leaf):
    keys, order = t.keys()
    sk = keys[order]
    nd = t.nodes()
    nn = t.n_nodes
    assert nd["level"][0] == 0 and nd["first"][0] == 0 and nd["count"][0] == len(m)
    # level-major, Morton order inside a level
    lv = nd["level"]
    assert np.all(np.diff(lv) >= 0)
    for L in np.unique(lv):
        sel = np.where(lv == L)[0]
        assert np.all(np.diff(nd["prefix"][sel].astype(np.int64)) > 0)
    for i in range(nn):
        L, s, c = int(lv[i]), int(nd["first"][i]), int(nd["count"][i])
        shift = np.uint64(3 * (21 - L))
        inside = (sk >> shift) == nd["prefix"][i]
        assert inside.sum() == c and inside[s:s + c].all()
        nc = int(nd["nchild"][i])
        if nc == 0:
            assert c <= n_leaf or L == 21
        else:
            assert c > n_leaf and L < 21
            cf = int(nd["child_first"][i])
            kids = np.arange(cf, cf + nc)
            assert np.all(nd["parent"][kids] == i)
            assert nd["first"][kids[0]] == s
            assert nd["count"][kids].sum() == c
            assert np.all(nd["first"][kids[1:]] == nd["first"][kids[:-1]] + nd["count"][kids[:-1]])
            assert np.all((nd["prefix"][kids] >> np.uint64(3)) == nd["prefix"][i])
        # geometry against numpy (exact max distance, weighted mean)
        X = pos[order[s:s + c]]
        w = m[order[s:s + c]]
        com = (w[:, None] * X).sum(0) / w.sum()
        np.testing.assert_allclose(nd["com"][i], com, rtol=1e-13, atol=1e-15)
        rmax = np.sqrt(((X - nd["com"][i]) ** 2).sum(1).max())
        assert abs(nd["rmax"][i] - rmax) <= 1e-14 * max(rmax, 1e-300)
        assert abs(nd["mass"][i] - w.sum()) <= 1e-14 * w.sum()
    return nd, order


def _check_walk(t, nd, order, n):
    far, near = t.lists()
    pos_of = np.empty(n, np.int64)
    pos_of[order] = np.arange(n)
    cover = np.zeros((n, n), np.int32)

    def members(i):
        return np.arange(nd["first"][i], nd["first"][i] + nd["count"][i])

    com, rmax = nd["com"], nd["rmax"]
    for a, b in far:
        assert a < b
        R = np.sqrt(((com[a] - com[b]) ** 2).sum())
        assert R > 0 and rmax[a] + rmax[b] <= t.theta * R
        ia, ib = members(a), members(b)
        assert not np.intersect1d(ia, ib).size
        cover[np.ix_(ia, ib)] += 1
        cover[np.ix_(ib, ia)] += 1
    for a, b in near:
        assert nd["nchild"][a] == 0 and nd["nchild"][b] == 0
        ia, ib = members(a), members(b)
        if a == b:
            cover[np.ix_(ia, ia)] += 1
        else:
            R = np.sqrt(((com[a] - com[b]) ** 2).sum())
            assert not (R > 0 and rmax[a] + rmax[b] <= t.theta * R)
            cover[np.ix_(ia, ib)] += 1
            cover[np.ix_(ib, ia)] += 1
    np.fill_diagonal(cover, 1)
    assert np.all(cover == 1)


@pytest.mark.parametrize("gen,n,n_leaf,theta", [
    ("plummer", 500, 8, 0.5), ("ball", 600, 16, 0.8), ("ball", 300, 1, 0.3),
    ("plummer", 400, 4, 0.0)])
def test_tree_and_walk_invariants(gen, n, n_leaf, theta):
    pos, m = (plummer if gen == "plummer" else uniform_ball)(n, 7)
    t = oracle.Tree(pos, m, n_leaf=n_leaf, theta=theta)
    nd, order = _check_nodes(t, pos, m, n_leaf)
    _check_walk(t, nd, order, n)


def test_degenerate_inputs():
    # single particle
    t = oracle.Tree(np.zeros((1, 3)), np.ones(1), n_leaf=4, theta=0.5)
    assert t.n_nodes == 1 and t.n_p2p == 1 and t.n_m2l == 0
    assert np.all(t.forces(4, 1e-3) == 0.0)
    # all particles coincident: ext = 0 -> 1, one level-21 leaf holding everything
    pos = np.full((40, 3), 0.25)
    m = np.full(40, 0.025)
    t = oracle.Tree(pos, m, n_leaf=4, theta=0.5)
    nd = t.nodes()
    assert t.bbox()[3] == 1.0
    assert nd["level"].max() == 21 and nd["count"][-1] == 40
    assert np.all(t.forces(2, 0.0) == 0.0)
    # duplicates mixed with distinct points, coplanar set
    rng = np.random.default_rng(3)
    pos = rng.random((200, 3))
    pos[:, 2] = 0.5
    pos[100:130] = pos[7]
    m = rng.uniform(0.5, 1.0, 200)
    t = oracle.Tree(pos, m, n_leaf=8, theta=0.6)
    nd, order = _check_nodes(t, pos, m, 8)
    _check_walk(t, nd, order, 200)
    d = oracle.diagnostics(pos, m, t.forces(3, 1e-2, "conserving"))
    assert d[18] < 1e-14 and d[19] < 1e-14


def test_invalid_arguments_are_rejected():
    pos, m = uniform_ball(10, 1)
    for kw in (dict(n_leaf=0, theta=0.5), dict(n_leaf=8, theta=1.0), dict(n_leaf=8, theta=-0.1)):
        with pytest.raises(ValueError):
            oracle.Tree(pos, m, **kw)
    t = oracle.Tree(pos, m, n_leaf=8, theta=0.5)
    with pytest.raises(ValueError):
        t.forces(0, 1e-3)
    with pytest.raises(ValueError):
        t.forces(9, 1e-3)
