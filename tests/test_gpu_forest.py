"""Forests (tfmm_build_forest, tfmm_forest_rebuild, tfmm_evaluate_forest):
several independent particle sets solved by one set of launches.

Each set must get exactly the tree, lists and forces it gets alone: the
forest keeps a bounding cube, a root and a walk start per set, and nothing
crosses sets, so the comparisons with the sets solved one at a time are
bitwise.  A few sets are also checked against the FP64 oracle.
"""

import ctypes

import numpy as np
import pytest

import oracle
from paper_2107_07166_amd.generators import generate
from parity import gate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_LEAF = 16

# (kind, n, seed, theta): sizes around and below n_leaf (one-leaf sets, a
# single particle), coincident points, a flat disk and a few thousand
# particles; thetas differ per set.
SETS = [("plummer", 5000, 11, 0.5), ("ball", 9, 12, 0.6), ("ball", 1, 13, 0.4),
        ("disk", 3000, 14, 0.8), ("same", 300, 15, 0.5), ("plummer", 2, 16, 0.7),
        ("ball", 12000, 17, 0.4), ("disk", 17, 18, 0.6), ("plummer", 700, 19, 0.3)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_07166_amd import api
    c = api.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _pairset(a):
    a = np.sort(np.asarray(a, dtype=np.int64).reshape(-1, 2), axis=1)
    return np.unique(a[:, 0] * (1 << 32) + a[:, 1])


def _make(kind, n, seed):
    if kind == "same":
        pos, m = generate("ball", n, seed)
        pos[: n // 2] = pos[0]          # half of the set at one point
        return pos, m
    return generate(kind, n, seed)


def _sets(specs):
    parts = [_make(k, n, s) for k, n, s, _ in specs]
    off = np.cumsum([0] + [len(m) for _, m in parts]).astype(np.int64)
    pos = np.concatenate([p for p, _ in parts])
    mass = np.concatenate([m for _, m in parts])
    return parts, off, pos, mass, np.array([th for *_, th in specs])


def _alone(ctx, parts, thetas, **kw):
    from paper_2107_07166_amd import api
    out = []
    for (p, m), th in zip(parts, thetas):
        pd, md = _dev(p), _dev(m)
        t = api.Tree(ctx, pd, md, n_leaf=N_LEAF)
        pot = torch.empty(len(m), dtype=torch.float64, device="cuda") if kw.get("with_pot") else None
        f = t.evaluate(theta=float(th), pot=pot, **{k: v for k, v in kw.items() if k != "with_pot"})
        out.append((f.cpu().numpy(), None if pot is None else pot.cpu().numpy(), t.export(), t.lists(), t.info()))
        t.close()
    return out


@pytest.mark.parametrize("p,variant,precision", [(4, "conserving", "mixed32"), (4, "standard", "fp64"),
                                                 (6, "conserving", "fp64"), (2, "standard", "mixed32"),
                                                 (1, "conserving_r2", "mixed32")])
def test_forest_forces_equal_sets_alone(ctx, p, variant, precision):
    from paper_2107_07166_amd import api
    parts, off, pos, mass, thetas = _sets(SETS)
    print(f"\n  forest of {len(parts)} sets, N={len(mass)}, p={p} {variant} {precision}", flush=True)
    kw = dict(p=p, eps=1e-3, variant=variant, precision=precision, G=1.3)
    alone = _alone(ctx, parts, thetas, with_pot=True, **kw)
    pd, md = _dev(pos), _dev(mass)
    t = api.Tree(ctx, pd, md, n_leaf=N_LEAF, offsets=off)
    pot = torch.empty(len(mass), dtype=torch.float64, device="cuda")
    f = t.evaluate_forest(thetas, pot=pot, **kw).cpu().numpy()
    pot = pot.cpu().numpy()
    info = t.info()
    assert info["nodes"] == sum(a[4]["nodes"] for a in alone)
    assert info["leaves"] == sum(a[4]["leaves"] for a in alone)
    assert info["far_pairs"] == sum(a[4]["far_pairs"] for a in alone)
    assert info["near_pairs"] == sum(a[4]["near_pairs"] for a in alone)
    for k, (fa, pa, *_) in enumerate(alone):
        assert np.array_equal(f[off[k]:off[k + 1]], fa), (k, "force")
        assert np.array_equal(pot[off[k]:off[k + 1]], pa), (k, "potential")
    t.close()


def test_forest_tree_and_lists_equal_sets_alone(ctx):
    """Node tables and interaction lists: the forest's nodes of set k, in id
    order, are the set's own tree renumbered."""
    from paper_2107_07166_amd import api
    parts, off, pos, mass, thetas = _sets(SETS)
    alone = _alone(ctx, parts, thetas, p=3, eps=1e-3, variant="standard", precision="fp64")
    t = api.Tree(ctx, _dev(pos), _dev(mass), n_leaf=N_LEAF, offsets=off)
    t.evaluate_forest(thetas, p=3, eps=1e-3, variant="standard", precision="fp64")
    g = t.export()
    far, near = t.lists()
    owner = np.searchsorted(off, g["first"], side="right") - 1   # set of every forest node
    assert np.array_equal(np.flatnonzero(g["level"] == 0), np.arange(len(parts)))  # root k is node k
    for k, (_, _, e, (fa, na), _) in enumerate(alone):
        ids = np.flatnonzero(owner == k)
        remap = np.full(len(g["level"]), -1, np.int64)
        remap[ids] = np.arange(len(ids))
        assert len(ids) == len(e["level"]), k
        assert np.array_equal(g["order"][off[k]:off[k + 1]] - off[k], e["order"]), k
        assert np.array_equal(g["keys"][off[k]:off[k + 1]], e["keys"]), k
        for name in ("level", "prefix", "count", "nchild", "com", "mass", "rmax"):
            assert np.array_equal(g[name][ids], e[name]), (k, name)
        assert np.array_equal(g["first"][ids] - off[k], e["first"]), k
        par = g["parent"][ids]
        assert np.array_equal(np.where(par < 0, -1, remap[np.maximum(par, 0)]), e["parent"]), k
        cf = g["child_first"][ids]
        assert np.array_equal(np.where(cf < 0, -1, remap[np.maximum(cf, 0)]), e["child_first"]), k
        for got, ref in ((far, fa), (near, na)):
            mine = got[owner[got[:, 0]] == k]
            assert np.all(owner[mine[:, 1]] == k), k   # no pair crosses sets
            assert np.array_equal(_pairset(remap[mine]), _pairset(ref)), k
    t.close()


def test_forest_matches_oracle(ctx):
    """Three sets of the forest against the oracle's trees of the sets alone."""
    from paper_2107_07166_amd import api
    specs = [("plummer", 4000, 31, 0.5), ("disk", 2500, 32, 0.8), ("ball", 6000, 33, 0.6)]
    parts, off, pos, mass, thetas = _sets(specs)
    t = api.Tree(ctx, _dev(pos), _dev(mass), n_leaf=N_LEAF, offsets=off)
    for variant in ("standard", "conserving"):
        for prec in ("fp64", "mixed32"):
            f = t.evaluate_forest(thetas, p=4, eps=1e-3, variant=variant, precision=prec).cpu().numpy()
            for k, ((p, m), th) in enumerate(zip(parts, thetas)):
                ot = oracle.Tree(p, m, n_leaf=N_LEAF, theta=float(th))
                sample = np.random.default_rng(k).choice(len(m), 400, replace=False)
                ref = ot.forces(4, 1e-3, variant, targets=sample)
                gate(f[off[k]:off[k + 1]][sample], ref, prec, f"forest set {k} {variant}")
    t.close()


def test_forest_uniform_theta_and_rebuilds(ctx):
    """tfmm_evaluate_forces on a forest uses params.theta for every set; a
    tree rebuilt as a forest, as another forest and back as one set gives
    what fresh trees give."""
    from paper_2107_07166_amd import api
    parts, off, pos, mass, _ = _sets(SETS)
    pd, md = _dev(pos), _dev(mass)
    kw = dict(p=4, eps=1e-3, variant="conserving", precision="mixed32")
    t = api.Tree(ctx, pd, md, n_leaf=N_LEAF, offsets=off)
    fa = t.evaluate(theta=0.55, **kw).cpu().numpy()
    fb = t.evaluate_forest(np.full(len(parts), 0.55), **kw).cpu().numpy()
    assert np.array_equal(fa, fb)
    # reuse: a different forest (the sets in reverse order), then one set
    rev = SETS[::-1]
    parts2, off2, pos2, mass2, th2 = _sets(rev)
    t.rebuild(_dev(pos2), _dev(mass2), offsets=off2)
    f2 = t.evaluate_forest(th2, **kw).cpu().numpy()
    fresh = api.Tree(ctx, _dev(pos2), _dev(mass2), n_leaf=N_LEAF, offsets=off2)
    assert np.array_equal(f2, fresh.evaluate_forest(th2, **kw).cpu().numpy())
    fresh.close()
    t.rebuild(pd, md)
    assert t.n_sets == 1
    f1 = t.evaluate(theta=0.5, **kw).cpu().numpy()
    one = api.Tree(ctx, pd, md, n_leaf=N_LEAF)
    assert np.array_equal(f1, one.evaluate(theta=0.5, **kw).cpu().numpy())
    one.close()
    t.close()


def test_forest_argument_errors(ctx):
    from paper_2107_07166_amd import _lib, api
    lib = ctx.lib
    pos, mass = generate("ball", 100, 3)
    pd, md = _dev(pos), _dev(mass)

    def build(off):
        a = np.asarray(off, dtype=np.int64)
        h = ctypes.c_void_p()
        rc = lib.tfmm_build_forest(ctx.handle, len(a) - 1, a.ctypes.data_as(ctypes.c_void_p), pd.data_ptr(),
                                   md.data_ptr(), 8, None, ctypes.byref(h))
        if rc == _lib.OK:
            lib.tfmm_tree_destroy(h)
        return rc

    assert build([0, 40, 100]) == _lib.OK
    assert build([1, 40, 100]) == _lib.EINVAL      # does not start at 0
    assert build([0, 40, 40, 100]) == _lib.EINVAL  # empty set
    assert build([0, 60, 40, 100]) == _lib.EINVAL  # not ascending
    assert build([0]) == _lib.EINVAL               # no set
    big = np.arange(0, 4098, dtype=np.int64)       # 4097 sets of one particle
    assert build(big) == _lib.EINVAL
    assert "4096" in lib.tfmm_last_error(ctx.handle).decode()
    t = api.Tree(ctx, pd, md, n_leaf=8, offsets=[0, 40, 100])
    with pytest.raises(api.TfmmError, match="theta"):
        t.evaluate_forest([0.5, 1.0])
    with pytest.raises(ValueError):
        t.evaluate_forest([0.5])
    f = torch.empty_like(pd)
    vel = torch.zeros_like(pd)
    prm = _lib.Params(4, 0.5, 1e-3, 1.0, _lib.CONSERVING, _lib.MIXED32, 0)
    rc = lib.tfmm_leapfrog(t.handle, ctypes.byref(prm), pd.data_ptr(), vel.data_ptr(), md.data_ptr(),
                           f.data_ptr(), 1e-3, 1, 0, None)
    assert rc == _lib.EINVAL and "one particle set" in lib.tfmm_last_error(ctx.handle).decode()
    t.close()


def test_forest_of_many_small_sets(ctx):
    """4096 sets (the limit; the sort by set takes two 8-bit passes) of 1 to
    40 particles: every set alone and in the forest give the same forces."""
    from paper_2107_07166_amd import api
    rng = np.random.default_rng(77)
    sizes = rng.integers(1, 41, 4096)
    specs = [("ball", int(n), 1000 + k, float(rng.choice([0.3, 0.5, 0.7]))) for k, n in enumerate(sizes)]
    parts, off, pos, mass, thetas = _sets(specs)
    kw = dict(p=3, eps=1e-3, variant="conserving", precision="mixed32")
    t = api.Tree(ctx, _dev(pos), _dev(mass), n_leaf=N_LEAF, offsets=off)
    f = t.evaluate_forest(thetas, **kw).cpu().numpy()
    assert t.info()["nodes"] >= 4096
    t.close()
    for k in rng.choice(4096, 24, replace=False):
        (p, m), th = parts[k], thetas[k]
        one = api.Tree(ctx, _dev(p), _dev(m), n_leaf=N_LEAF)
        fa = one.evaluate(theta=float(th), **kw).cpu().numpy()
        one.close()
        assert np.array_equal(f[off[k]:off[k + 1]], fa), k


def test_forest_with_scalar_degree(ctx):
    """The scalar-degree knob (locals of order K + 1) on a forest equals the
    sets alone."""
    from paper_2107_07166_amd import api
    parts, off, pos, mass, thetas = _sets(SETS[:6])
    kw = dict(p=3, eps=1e-3, variant="conserving", precision="fp64", scalar_degree=4)
    alone = _alone(ctx, parts, thetas, **kw)
    t = api.Tree(ctx, _dev(pos), _dev(mass), n_leaf=N_LEAF, offsets=off)
    f = t.evaluate_forest(thetas, **kw).cpu().numpy()
    t.close()
    for k, (fa, *_) in enumerate(alone):
        assert np.array_equal(f[off[k]:off[k + 1]], fa), k


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_random_forests_equal_sets_alone(ctx, seed):
    """Seeded random forests: 2 to 40 sets of 1 to 3000 particles from every
    generator, per-set thetas, a random order, variant and precision; each
    set's forces equal its forces alone bit for bit."""
    from paper_2107_07166_amd import api
    rng = np.random.default_rng(900 + seed)
    k = int(rng.integers(2, 41))
    specs = [(str(rng.choice(["ball", "plummer", "disk", "same"])), int(rng.integers(1, 3001)),
              int(rng.integers(1 << 20)), float(rng.choice([0.0, 0.3, 0.5, 0.7, 0.9]))) for _ in range(k)]
    p = int(rng.integers(1, 8))
    variant = str(rng.choice(["standard", "conserving"]))
    precision = str(rng.choice(["fp64", "mixed32"]))
    n_leaf = int(rng.choice([1, 4, 16, 64]))
    print(f"\n  seed {seed}: {k} sets, p={p} {variant} {precision} n_leaf={n_leaf}", flush=True)
    parts, off, pos, mass, thetas = _sets(specs)
    kw = dict(p=p, eps=float(rng.choice([0.0, 1e-3])), variant=variant, precision=precision)
    t = api.Tree(ctx, _dev(pos), _dev(mass), n_leaf=n_leaf, offsets=off)
    f = t.evaluate_forest(thetas, **kw).cpu().numpy()
    t.close()
    for j, ((pp, m), th) in enumerate(zip(parts, thetas)):
        one = api.Tree(ctx, _dev(pp), _dev(m), n_leaf=n_leaf)
        fa = one.evaluate(theta=float(th), **kw).cpu().numpy()
        one.close()
        assert np.array_equal(f[off[j]:off[j + 1]], fa), j
