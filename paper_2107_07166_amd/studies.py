"""Measurement studies beyond the headline benchmark (one JSON line each).

    python -m paper_2107_07166_amd.studies binary [--n N] [--steps 200] [--dt 1e-3]
        Two n=1 polytropes on a circular orbit (p=4, theta=0.7, mixed): the
        angular momentum drift of the standard and the conserving variant over
        leapfrog steps, the relative energy change over the run, and the time
        per step.
    python -m paper_2107_07166_amd.studies disk [--n N]
        Exponential disk (p=6, theta=0.8): time of both variants (the cost of
        realignment), net torque, mixed vs FP64 force difference.
    python -m paper_2107_07166_amd.studies serve [--requests 512] [--sessions 16]
        Poisson trace of solves with N log-uniform in [1e3, 5e5], p in {2,4,6},
        theta in {0.4,0.6,0.8}, plus persistent leapfrog sessions: FP32 mixed
        with concurrent slots against FP64 one solve at a time, same trace;
        solves/s and p50/p99 latency, the per-request mixed-vs-FP64 error, and
        the capacity of both (the same solves queued at once, no sessions).
    python -m paper_2107_07166_amd.studies profile [--steps 3] [--n-leaf 64]
                                                   [--workload plummer1m] [--variant conserving]
        Driver for profilers: a workload (default the benchmark one, Plummer
        N=2^20, p=4, theta=0.5; mixed precision), one tree, then --steps
        rebuild + walk + evaluate steps with per-phase event times.
    python -m paper_2107_07166_amd.studies copy
        Counter calibration: three device copies of a 256 MiB buffer.
    python -m paper_2107_07166_amd.studies shapes [--n 4000]
        Two irregular bodies of n particles each at distances 3.6-16 (units of
        their radius), each body one leaf, theta = 0.99: error of the inter-body
        force for orders 0 and 1 with and without realignment (both
        realignments at order 0), net force and torque (FP64, eps = 0).
    python -m paper_2107_07166_amd.studies knob [--n-leaf 64] [--reps 5]
        The benchmark workload with the conserving projection scalar kept to
        degree K = p-1, p, p+1 (p = 2, 4, 5): time per evaluation, error
        against the p = 8 standard FP64 evaluation, net torque.
    python -m paper_2107_07166_amd.studies zeroth [--n-leaf 64] [--reps 5]
        The benchmark workload at orders 0 and 1 with and without
        realignment: time per evaluation, net torque, error against p = 4.
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import time

import numpy as np
import torch

from . import api, generators


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def study_binary(n: int, steps: int, dt: float, n_leaf: int) -> dict:
    from .session import Session
    w = generators.WORKLOADS["binary4m"]
    pos, mass, vel = w.make(n=n, velocities=True)
    out = {"study": "binary", "n": n, "p": w.p, "theta": w.theta, "dt": dt, "steps": steps, "n_leaf": n_leaf}
    for variant in ("standard", "conserving"):
        ctx = api.Context(0)
        s = Session(ctx, _dev(pos), _dev(vel), _dev(mass), p=w.p, theta=w.theta, eps=w.eps, variant=variant,
                    precision="mixed32", n_leaf=n_leaf)
        d0 = s.diagnostics()
        L0 = d0["L"]
        E0 = s.energy()["E"]
        drift, torque = [], []
        t_total = 0.0
        for k in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(dt, 1)
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t0
            d = s.diagnostics()
            drift.append(float(np.linalg.norm(d["L"] - L0) / np.linalg.norm(L0)))
            torque.append(d["torque_rel"])
        E1 = s.energy()["E"]
        out[variant] = {"L_drift_final": drift[-1], "L_drift_max": max(drift),
                        "L_drift_every_20": drift[19::20], "torque_rel_mean": float(np.mean(torque)),
                        "P_final": [float(x) for x in d["P"]], "ms_per_step": 1e3 * t_total / steps,
                        "E0": E0, "E_drift_final": abs(E1 - E0) / abs(E0)}
        s.close()
        ctx.close()
    return out


def study_disk(n: int, n_leaf: int, reps: int) -> dict:
    w = generators.WORKLOADS["disk4m"]
    pos, mass = w.make(n=n)
    pd, md = _dev(pos), _dev(mass)
    ctx = api.Context(0)
    tree = api.Tree(ctx, pd, md, n_leaf=n_leaf)
    out = {"study": "disk", "n": n, "p": w.p, "theta": w.theta, "n_leaf": n_leaf}
    forces = {}
    for variant in ("standard", "conserving"):
        for prec in ("mixed32", "fp64"):
            f = tree.evaluate(p=w.p, theta=w.theta, eps=w.eps, variant=variant, precision=prec)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                tree.rebuild(pd, md)
                tree.evaluate(p=w.p, theta=w.theta, eps=w.eps, variant=variant, precision=prec, out=f)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            d = ctx.diagnostics(pd, md, f)
            forces[variant, prec] = f.cpu().numpy()
            out[f"{variant}_{prec}"] = {"ms": 1e3 * float(np.median(ts)), "torque_rel": float(d[19]),
                                         "force_rel": float(d[18]), "evals_per_s": n / float(np.median(ts))}
    for variant in ("standard", "conserving"):
        a, b = forces[variant, "mixed32"], forces[variant, "fp64"]
        out[f"{variant}_mixed_vs_fp64_rms"] = float(np.sqrt(np.mean(((a - b) ** 2).sum(1) / (b ** 2).sum(1))))
    out["conserving_overhead_mixed"] = out["conserving_mixed32"]["ms"] / out["standard_mixed32"]["ms"] - 1.0
    out["tree"] = tree.info()
    tree.close()
    ctx.close()
    return out


def study_serve(n_requests: int, n_sessions: int, rate: float, slots: int, budget_gb: float) -> dict:
    from .serve import Server, close_sessions, make_inputs, make_sessions, make_trace, summarize
    trace = make_trace(n_requests, rate=rate)
    inputs = {r.rid: make_inputs(r) for r in trace}
    out = {"study": "serve", "requests": n_requests, "sessions": n_sessions, "rate_per_s": rate, "slots": slots,
           "budget_GB": budget_gb}
    res = {}
    for name, prec, k in (("fp64_one_at_a_time", "fp64", 1), ("mixed32_batched", "mixed32", slots)):
        sessions = make_sessions(n_sessions, precision=prec)
        try:
            recs = Server(slots=k, precision=prec, budget_bytes=int(budget_gb * (1 << 30))).run(
                trace, sessions=sessions, inputs=inputs)
        finally:
            close_sessions(sessions)
        res[name] = recs
        out[name] = summarize(recs)
    # capacity: the same solves all queued at once, no sessions
    burst = [dataclasses.replace(r, arrival=0.0) for r in trace]
    for name, prec, k in (("fp64_one_at_a_time", "fp64", 1), ("mixed32_batched", "mixed32", slots)):
        recs = Server(slots=k, precision=prec, budget_bytes=int(budget_gb * (1 << 30))).run(burst, inputs=inputs)
        out[name]["capacity_solves_per_s"] = summarize(recs)["solves_per_s"]
    a = {r.rid: r.sample for r in res["mixed32_batched"] if r.kind == "solve" and not r.error}
    b = {r.rid: r.sample for r in res["fp64_one_at_a_time"] if r.kind == "solve" and not r.error}
    errs = [float(np.sqrt(np.mean(((a[i] - b[i]) ** 2).sum(1) / (b[i] ** 2).sum(1)))) for i in a if i in b]
    out["mixed_vs_fp64_rms_per_request"] = {"max": max(errs), "median": float(np.median(errs))}
    return out


def study_profile(steps: int, n_leaf: int, workload: str = "plummer1m", variant: str = "conserving") -> dict:
    w = generators.WORKLOADS[workload]
    pos, mass = w.make()
    pd, md = _dev(pos), _dev(mass)
    ctx = api.Context(0)
    tree = api.Tree(ctx, pd, md, n_leaf=n_leaf)
    f = torch.empty((w.n, 3), dtype=torch.float64, device=pd.device)
    tree.set_timing(True)
    for _ in range(steps):
        tree.rebuild(pd, md)
        tree.evaluate(p=w.p, theta=w.theta, eps=w.eps, variant=variant, precision="mixed32", out=f)
    torch.cuda.synchronize()
    out = {"study": "profile", "workload": workload, "variant": variant, "steps": steps, "n_leaf": n_leaf,
           "tree": tree.info(),
           "phases_ms_mean": tree.phase_times()}
    tree.close()
    ctx.close()
    return out


SHAPE_CASES = (("order0", 1, "standard"), ("order0_realigned_r2", 1, "conserving_r2"),
               ("order0_projected", 1, "conserving"), ("order1", 2, "standard"),
               ("order1_realigned", 2, "conserving"))


def _rel_rms(err, ref):
    return float(np.sqrt(np.mean((err * err).sum(1) / (ref * ref).sum(1))))


def study_shapes(n_each: int, seps, seed: int) -> dict:
    """Two irregular bodies at a varying distance (in units of their radius),
    each body one leaf (n_leaf = n_each) and theta = 0.99, so the only far
    interaction is the one body-body node pair, FP64, eps = 0.  Error of the
    inter-body force per particle (relative to the exact inter-body force,
    rms over both bodies) for orders 0 and 1 with and without realignment,
    plus the net force and torque of the whole evaluation."""
    ctx = api.Context(0)
    rows = []
    for sep in seps:
        pos, mass = generators.irregular_pair(n_each, seed, sep)
        t = api.Tree(ctx, _dev(pos), _dev(mass), n_leaf=n_each)
        exact = t.evaluate(p=1, theta=0.0, eps=0.0, variant="standard", precision="fp64").cpu().numpy()
        alone = []
        for half in (slice(0, n_each), slice(n_each, 2 * n_each)):
            ta = api.Tree(ctx, _dev(pos[half]), _dev(mass[half]), n_leaf=n_each)
            alone.append(ta.evaluate(p=1, theta=0.0, eps=0.0, variant="standard", precision="fp64").cpu().numpy())
            ta.close()
        inter = exact - np.concatenate(alone)
        row = {"separation": sep}
        for label, p, variant in SHAPE_CASES:
            ft = t.evaluate(p=p, theta=0.99, eps=0.0, variant=variant, precision="fp64")
            d = ctx.diagnostics(_dev(pos), _dev(mass), ft)
            f = ft.cpu().numpy()
            row[label] = {"err": _rel_rms(f - exact, inter), "net_force_rel": float(d[18]),
                          "net_torque_rel": float(d[19])}
        info = t.info()
        row["far_pairs"] = info["far_pairs"]
        row["leaves"] = info["leaves"]
        rows.append(row)
        t.close()
    ctx.close()
    return {"study": "shapes", "n_each": n_each, "seed": seed, "theta": 0.99, "rows": rows}


def study_zeroth(n_leaf: int, reps: int) -> dict:
    """The benchmark workload (Plummer N = 2^20, theta = 0.5, mixed) at orders
    0 and 1 with and without realignment: time per evaluation (tree and walk
    kept), net torque, and the rms error against the p = 4 conserving FP64
    evaluation of the same tree."""
    w = generators.WORKLOADS["plummer1m"]
    pos, mass = w.make()
    ctx = api.Context(0)
    pd, md = _dev(pos), _dev(mass)
    t = api.Tree(ctx, pd, md, n_leaf=n_leaf)
    ref = t.evaluate(p=4, theta=w.theta, eps=w.eps, variant="conserving", precision="fp64").cpu().numpy()
    out = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
    rows = {}
    for label, p, variant in SHAPE_CASES:
        t.evaluate(p=p, theta=w.theta, eps=w.eps, variant=variant, precision="mixed32", out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            t.evaluate(p=p, theta=w.theta, eps=w.eps, variant=variant, precision="mixed32", out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        d = ctx.diagnostics(pd, md, out)
        rows[label] = {"p": p, "variant": variant, "ms_per_eval": ms,
                       "err_vs_p4_fp64": _rel_rms(out.cpu().numpy() - ref, ref),
                       "net_torque_rel": float(d[19])}
    t.close()
    ctx.close()
    return {"study": "zeroth", "workload": w.name, "n_leaf": n_leaf, "theta": w.theta, "rows": rows}


def study_orders(n_leaf: int, reps: int, orders=(2, 3, 4, 5, 6, 8)) -> dict:
    """The benchmark workload (Plummer N = 2^20, theta = 0.5, mixed) at several
    orders p, standard and conserving: time per evaluation (tree and walk
    kept), the conserving variant's overhead, net torque, and the rms error
    against the p = 8 conserving FP64 evaluation of the same tree."""
    w = generators.WORKLOADS["plummer1m"]
    pos, mass = w.make()
    ctx = api.Context(0)
    pd, md = _dev(pos), _dev(mass)
    t = api.Tree(ctx, pd, md, n_leaf=n_leaf)
    ref = t.evaluate(p=8, theta=w.theta, eps=w.eps, variant="conserving", precision="fp64").cpu().numpy()
    out = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
    rows = {}
    for p in orders:
        row = {}
        for variant in ("standard", "conserving"):
            t.evaluate(p=p, theta=w.theta, eps=w.eps, variant=variant, precision="mixed32", out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                t.evaluate(p=p, theta=w.theta, eps=w.eps, variant=variant, precision="mixed32", out=out)
            torch.cuda.synchronize()
            d = ctx.diagnostics(pd, md, out)
            row[variant] = {"ms_per_eval": (time.perf_counter() - t0) / reps * 1e3,
                            "err_vs_p8_fp64": _rel_rms(out.cpu().numpy() - ref, ref),
                            "net_torque_rel": float(d[19])}
        row["conserving_overhead"] = row["conserving"]["ms_per_eval"] / row["standard"]["ms_per_eval"] - 1.0
        rows[str(p)] = row
    t.close()
    ctx.close()
    return {"study": "orders", "workload": w.name, "n_leaf": n_leaf, "theta": w.theta, "rows": rows}


def study_knob(n_leaf: int, reps: int) -> dict:
    """The benchmark workload (Plummer N = 2^20, theta = 0.5, mixed) with the
    conserving projection scalar kept to degree K = p - 1, p, p + 1 for
    p = 2, 4, 5: time per evaluation (tree and walk kept), rms error against
    the p = 8 standard FP64 evaluation, net torque; the standard variant of
    the same p beside it."""
    w = generators.WORKLOADS["plummer1m"]
    pos, mass = w.make()
    pd, md = _dev(pos), _dev(mass)
    ctx = api.Context(0)
    tree = api.Tree(ctx, pd, md, n_leaf=n_leaf)
    ref = tree.evaluate(p=8, theta=w.theta, eps=w.eps, variant="standard", precision="fp64").cpu().numpy()
    rows = []
    for p in (2, 4, 5):
        cases = [("standard", 0)] + [("conserving", k) for k in range(p - 1, min(p + 1, 6) + 1)]
        for variant, k in cases:
            kw = dict(p=p, theta=w.theta, eps=w.eps, variant=variant, precision="mixed32", scalar_degree=k)
            f = tree.evaluate(**kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                tree.evaluate(out=f, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            d = ctx.diagnostics(pd, md, f)
            rows.append({"p": p, "variant": variant, "K": k if variant == "conserving" else None, "ms": ms,
                         "err_vs_p8": _rel_rms(f.cpu().numpy() - ref, ref), "net_torque_rel": float(d[19])})
    tree.close()
    ctx.close()
    return {"study": "knob", "workload": "plummer1m", "n_leaf": n_leaf, "rows": rows}


def study_copy() -> dict:
    x = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"study": "copy", "bytes_per_copy": 256 << 20, "copies": 3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["binary", "disk", "serve", "profile", "copy", "shapes", "zeroth", "orders",
                                      "knob"])
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--n-leaf", type=int, default=32)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--sessions", type=int, default=16)
    ap.add_argument("--rate", type=float, default=100.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--workload", default="plummer1m", choices=sorted(generators.WORKLOADS))
    ap.add_argument("--variant", default="conserving", choices=["standard", "conserving"])
    a = ap.parse_args()
    if a.study == "binary":
        r = study_binary(a.n or (1 << 22), a.steps, a.dt, a.n_leaf)
    elif a.study == "disk":
        r = study_disk(a.n or 4194304, a.n_leaf, a.reps)
    elif a.study == "profile":
        r = study_profile(a.steps, a.n_leaf, a.workload, a.variant)
    elif a.study == "copy":
        r = study_copy()
    elif a.study == "shapes":
        r = study_shapes(a.n or 4000, (3.6, 4.0, 5.0, 6.0, 8.0, 12.0, 16.0), 210707170)
    elif a.study == "zeroth":
        r = study_zeroth(a.n_leaf, a.reps)
    elif a.study == "orders":
        r = study_orders(a.n_leaf, a.reps)
    elif a.study == "knob":
        r = study_knob(a.n_leaf, a.reps)
    else:
        r = study_serve(a.requests, a.sessions, a.rate, a.slots, a.budget_gb)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
