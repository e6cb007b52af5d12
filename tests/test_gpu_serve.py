"""Serving: continuous admission, memory budget, sessions, forests of small
requests, alone == in the mix."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def _reqs():
    from paper_2107_07166_amd.serve import Request
    specs = [(3000, "plummer", 2, 0.4, "standard"), (12000, "ball", 4, 0.6, "conserving"),
             (7000, "disk", 6, 0.8, "conserving"), (20000, "plummer", 4, 0.5, "standard"),
             (1500, "ball", 6, 0.4, "conserving"), (9000, "disk", 2, 0.8, "standard")]
    return [Request(rid=i, arrival=0.0, n=n, gen=g, seed=100 + i, p=p, theta=th, variant=v)
            for i, (n, g, p, th, v) in enumerate(specs)]


def test_alone_equals_in_the_mix(gpu):
    from paper_2107_07166_amd.serve import Server, make_trace, make_sessions, close_sessions
    base = _reqs()
    alone = {}
    for r in base:
        rec = Server(slots=1, keep_full=True).run([r])
        assert len(rec) == 1 and not rec[0].error
        alone[r.rid] = rec[0].full
    others = make_trace(12, rate=400.0, seed=5, n_min=1e3, n_max=3e4)
    for k, r in enumerate(others):
        r.rid = 100 + k
    sessions = make_sessions(2, n_min=2e3, n_max=8e3)
    try:
        recs = Server(slots=4, keep_full=True).run(base + others, sessions=sessions)
    finally:
        close_sessions(sessions)
    got = {r.rid: r.full for r in recs if r.kind == "solve"}
    assert all(not r.error for r in recs)
    assert sum(1 for r in recs if r.kind == "step") > 0
    # requests of the same order and variant were solved together in forests
    assert max(r.batch for r in recs if r.kind == "solve") > 1
    for r in base:
        assert np.array_equal(got[r.rid], alone[r.rid]), r.rid


def test_memory_budget_queues_and_rejects(gpu):
    from paper_2107_07166_amd.serve import Server
    reqs = _reqs()
    srv = Server(slots=4)
    fps = sorted(srv.footprint(r) for r in reqs)
    # room for the largest request only: everything is served, one launch
    # set at a time (a forest of small requests that fits counts as one)
    srv_one = Server(slots=4, budget_bytes=fps[-1])
    recs = srv_one.run(reqs)
    assert all(not r.error for r in recs) and len(recs) == len(reqs)
    spans = sorted(set((r.admitted, r.done) for r in recs))
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-6  # never two launch sets at once under this budget
    # a budget below the largest footprint rejects it and serves the rest
    recs = Server(slots=4, budget_bytes=fps[-2]).run(reqs)
    bad = [r for r in recs if r.error]
    assert len(bad) == 1 and "budget" in bad[0].error
    assert sum(1 for r in recs if not r.error) == len(reqs) - 1


def test_memory_budget_counts_what_slots_hold(gpu):
    """Slots keep their trees, reusable blocks and request buffers between
    solves; the admission counts them, so under a budget of about two of the
    larger footprints the reservations never exceed the budget, and no slot
    ever holds more than it reserved (the library part is capped by the slot
    context's budget)."""
    from paper_2107_07166_amd.serve import Server, make_trace
    reqs = _reqs() + make_trace(16, rate=300.0, seed=13, n_min=2e3, n_max=6e4)
    for k, r in enumerate(reqs):
        r.rid = k
    probe = Server(slots=4)
    fps = sorted(probe.footprint(r) for r in reqs)
    budget = fps[-1] + fps[-2]
    srv = Server(slots=4, budget_bytes=budget, keep_full=True)
    recs = srv.run(reqs)
    assert all(not r.error for r in recs), [r.error for r in recs if r.error]
    assert len(recs) == len(reqs)
    assert srv.over_reservation == 0
    assert srv.peak_reserved <= budget
    # the same solves with an unlimited budget give the same forces
    free = {r.rid: r.full for r in Server(slots=4, keep_full=True).run(reqs)}
    for r in recs:
        assert np.array_equal(r.full, free[r.rid]), r.rid


def test_forest_batches_equal_requests_alone(gpu):
    """A burst of small requests: with forests (many requests per launch set)
    and without (batch_max_sets=1) every request gets the same forces."""
    from paper_2107_07166_amd.serve import Server, make_trace
    reqs = make_trace(40, rate=1e6, seed=21, n_min=500, n_max=2e4)
    for r in reqs:
        r.arrival = 0.0
    batched = Server(slots=2, keep_full=True).run(reqs)
    single = {r.rid: r.full for r in Server(slots=2, keep_full=True, batch_max_sets=1).run(reqs)}
    assert all(not r.error for r in batched)
    assert max(r.batch for r in batched) >= 4
    assert all(r.batch == 1 for r in Server(slots=1, batch_max_sets=1).run(reqs[:3]))
    for r in batched:
        assert np.array_equal(r.full, single[r.rid]), (r.rid, r.batch)
