"""GPU parity against the FP64 oracle on the named workloads at their full
sizes, the two-body setup of the paper's distance test, served requests and
the one-shot entry point (all through the C ABI).

* disk: exponential disk, N = 2^22, p = 6, theta = 0.8 (a wide acceptance
  angle at a high order);
* binary: two n = 1 polytropes of 2^21 particles each, p = 4, theta = 0.7;
* the distance test (Sec. 4, the force-error-against-distance figure): two
  irregular bodies of 4000 particles, each one leaf, theta = 0.99, eps = 0,
  orders 0 and 1 (p = 1, 2), with and without realignment.

Forces are compared on 1000 sampled particles per workload (the oracle sums
every particle pair of the accepted node pairs, so it is evaluated particle
by particle), with rms and per-particle max gates; net force and net torque
are checked on the full GPU result.
"""

import numpy as np
import pytest

import oracle
from paper_2107_07166_amd.generators import WORKLOADS, irregular_pair
from parity import gate, gate_momenta

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_SAMPLE = 1000


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
    a = np.asarray(a, dtype=np.int64).reshape(-1, 2)
    return np.unique(a[:, 0] * (1 << 32) + a[:, 1])


@pytest.mark.parametrize("name", ["disk4m", "binary4m"])
def test_full_size_workload(ctx, name):
    """Tree and lists bit-exact; sampled forces of both variants in both
    precisions against the oracle; momenta of the full result."""
    from paper_2107_07166_amd import api
    w = WORKLOADS[name]
    print(f"\n  {name}: N={w.n} p={w.p} theta={w.theta}", flush=True)
    pos, m = w.make()
    ot = oracle.Tree(pos, m, n_leaf=64, theta=w.theta)
    pd, md = _dev(pos), _dev(m)
    gt = api.Tree(ctx, pd, md, n_leaf=64)
    g = gt.export()
    ok, oo = ot.keys()
    assert np.array_equal(g["keys"], ok) and np.array_equal(g["order"].astype(np.int64), oo)
    on = ot.nodes()
    for k in ("level", "first", "count", "parent"):
        assert np.array_equal(g[k].astype(np.int64), on[k].astype(np.int64)), k
    for k in ("com", "rmax"):
        assert np.array_equal(g[k], on[k]), k
    gt.walk(w.theta)
    gf, gn = gt.lists()
    of, onr = ot.lists()
    assert np.array_equal(_pairset(gf), _pairset(of))
    assert np.array_equal(_pairset(gn), _pairset(onr))
    sample = np.random.default_rng(3).choice(w.n, N_SAMPLE, replace=False)
    for variant in ("standard", "conserving"):
        ref = ot.forces(w.p, w.eps, variant, targets=sample)
        for prec in ("fp64", "mixed32"):
            ft = gt.evaluate(p=w.p, theta=w.theta, eps=w.eps, variant=variant, precision=prec)
            gate_momenta(ctx.diagnostics(pd, md, ft), prec, variant, name)
            gate(ft.cpu().numpy()[sample], ref, prec, f"{name} {variant}")
    gt.close()


@pytest.mark.parametrize("sep", [3.6, 8.0, 16.0])
def test_distance_test_setup(ctx, sep):
    """The two-body setup of the distance figure: exactly one far pair (the
    two bodies), near field inside each body; orders 0 and 1, standard,
    realigned (Eq. realign; Eq. aaB1 at order 1) and, at order 0, realigned by
    magnitude (Eq. realign2 / aaB0).  Every particle is compared."""
    from paper_2107_07166_amd import api
    pos, m = irregular_pair(4000, 5, sep)
    ot = oracle.Tree(pos, m, n_leaf=4000, theta=0.99)
    assert ot.n_m2l == 1
    pd, md = _dev(pos), _dev(m)
    gt = api.Tree(ctx, pd, md, n_leaf=4000)
    gt.walk(0.99)
    assert gt.info()["far_pairs"] == 1
    for p, variant in ((1, "standard"), (1, "conserving"), (1, "conserving_r2"), (2, "standard"),
                       (2, "conserving")):
        ref = ot.forces(p, 0.0, variant)
        for prec in ("fp64", "mixed32"):
            ft = gt.evaluate(p=p, theta=0.99, eps=0.0, variant=variant, precision=prec)
            gate_momenta(ctx.diagnostics(pd, md, ft), prec, variant, f"two-body d={sep} p={p}")
            gate(ft.cpu().numpy(), ref, prec, f"two-body d={sep} p={p} {variant}")
    gt.close()


def test_served_requests_match_oracle(ctx):
    """Three requests served in a mix with others (four slots, two sessions),
    each solved in a forest with a companion of the same order and variant,
    return the oracle's forces for their own particle sets."""
    from paper_2107_07166_amd import generators
    from paper_2107_07166_amd.serve import Request, Server, close_sessions, make_sessions, make_trace
    mine = [Request(rid=0, arrival=0.0, n=12000, gen="plummer", seed=501, p=4, theta=0.6, variant="conserving"),
            Request(rid=1, arrival=0.0, n=7000, gen="disk", seed=502, p=6, theta=0.8, variant="standard"),
            Request(rid=2, arrival=0.0, n=3000, gen="ball", seed=503, p=2, theta=0.4, variant="conserving")]
    mates = [Request(rid=10 + k, arrival=0.0, n=2000 + 500 * k, gen="ball", seed=510 + k, p=r.p, theta=0.5,
                     variant=r.variant) for k, r in enumerate(mine)]
    mine_and_mates = [x for pair in zip(mine, mates) for x in pair]
    others = make_trace(10, rate=400.0, seed=9, n_min=1e3, n_max=2e4)
    for k, r in enumerate(others):
        r.rid = 100 + k
    sessions = make_sessions(2, n_min=2e3, n_max=6e3)
    try:
        srv = Server(slots=4, keep_full=True)
        recs = srv.run(mine_and_mates + others, sessions=sessions)
    finally:
        close_sessions(sessions)
    got = {r.rid: r for r in recs if r.kind == "solve"}
    assert all(not r.error for r in recs)
    assert all(got[r.rid].batch > 1 for r in mine), [got[r.rid].batch for r in mine]
    for r in mine:
        pos, m = generators.generate(r.gen, r.n, r.seed)
        ref = oracle.Tree(pos, m, n_leaf=srv.n_leaf, theta=r.theta).forces(r.p, r.eps, r.variant)
        gate(got[r.rid].full, ref, srv.precision, f"served {r.gen} n={r.n} p={r.p} {r.variant}")


@pytest.mark.parametrize("variant,prec", [("conserving", "mixed32"), ("standard", "fp64")])
def test_oneshot_equals_build_and_evaluate(ctx, variant, prec):
    """tfmm_evaluate_forces_oneshot builds, evaluates and destroys a tree in
    one call: bit-identical to tfmm_build_tree + tfmm_evaluate_forces."""
    from paper_2107_07166_amd import api
    pos, m = WORKLOADS["plummer1m"].make(n=50000)
    pd, md = _dev(pos), _dev(m)
    f1 = api.evaluate_forces_oneshot(pd, md, p=4, theta=0.5, eps=1e-3, variant=variant, precision=prec,
                                     n_leaf=32, ctx=ctx).cpu().numpy()
    gt = api.Tree(ctx, pd, md, n_leaf=32)
    f2 = gt.evaluate(p=4, theta=0.5, eps=1e-3, variant=variant, precision=prec).cpu().numpy()
    gt.close()
    assert np.array_equal(f1, f2)
    sample = np.random.default_rng(4).choice(len(m), 300, replace=False)
    ref = oracle.Tree(pos, m, n_leaf=32, theta=0.5).forces(4, 1e-3, variant, targets=sample)
    gate(f1[sample], ref, prec, f"oneshot {variant}")
