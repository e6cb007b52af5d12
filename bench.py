"""Benchmark: particle force evaluations per second on one MI355X.

Headline workload: Plummer sphere, N = 2^20 equal masses (total 1), scale
radius 1, softening 1e-3, expansion order p = 4, theta = tan(theta_MAC) = 0.5,
seeded synthetic input resident in HBM.  One step = one full force
evaluation of the conserving (torque-free) variant in the mixed path: tree
rebuild (keys, sort, octree, centres of mass, r_max), walk, moments, M2L,
L2L, P2P, L2P.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Besides the headline value it reports:

* the standard variant and the FP64 path at the same workload (every variant
  timed the same way: K steps after W warm-up steps);
* per-phase device times (rebuild, walk, moments, M2L, P2P, L2L, L2P, the
  interaction pass where P2P and M2L run side by side) from K further steps
  with the library's per-phase HIP events on;
* the roofline of the dominant kernel (P2P) and the algorithmic FLOP rate of
  the whole interaction pass (P2P + M2L);
* the exponential disk (N = 2^22, p = 6, theta = 0.8): ms per step of both
  variants and the conserving overhead;
* a bounded serving run: Poisson-arriving solves of N log-uniform in
  [1e3, 5e5], p in {2,4,6}, theta in {0.4,0.6,0.8}, plus resident leapfrog
  sessions; FP64 one solve at a time, mixed precision on several slots, and
  the same slots with requests of up to 2e5 particles solved together as
  forests, on the same
  trace: solves/s at capacity (the trace four times over, queued at once),
  p50/p99 latency at a fixed arrival rate;
* the two-body setup of the paper's distance test: force error of orders 0
  and 1 with and without realignment;
* the CPU oracle timed on a bounded sample of the headline workload.
"""

from __future__ import annotations

import argparse
import dataclasses
import importlib.util
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_FP32_NOPK_TFLOPS = 78.6  # the same without packed FP32 (256 CU x 64 FMA/clk x 2 x 2.4 GHz)
P2P_FLOP_PER_PAIR = 20        # per directed particle interaction (convention)

# HBM bytes per P2P launch at this workload, from rocprofv3 FETCH_SIZE (x2, the
# factor a plain copy of known size reads) and WRITE_SIZE (x1); see
# profiles/p2p_plummer1m_counters.md.  Valid only for the kernel source the
# counters were taken with (first 16 hex digits of its sha256).
P2P_TRAFFIC_BYTES = (2 * 141322 + 32239) * 1024
P2P_TRAFFIC_SOURCE_SHA = "21e0660b9e0ee718"


def _p2p_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2107_07166_amd", "csrc", "p2p.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return P2P_TRAFFIC_BYTES if sha == P2P_TRAFFIC_SOURCE_SHA else None


def _m2l_pair_flops(p, variant):
    """Algorithmic FLOPs per directed far pair, counted in the generated code."""
    path = os.path.join(ROOT, "paper_2107_07166_amd", "csrc", "gen_expansions.py")
    spec = importlib.util.spec_from_file_location("gen_expansions", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.pair_flops(p, variant)


def _erms(f, ref):
    return float(np.sqrt(np.mean(((f - ref) ** 2).sum(1) / (ref ** 2).sum(1))))


def _timed_steps(tree, pd, md, out, w, variant, precision, steps, warmup):
    """K timed steps (rebuild + evaluate) after W warm-up steps, then K more
    with the library's phase events on (the events cost a few per cent of a
    step of their own, so they stay out of the timed steps); returns
    (seconds per step, phase times).  Every variant is timed this way."""
    import torch

    def step():
        tree.rebuild(pd, md)
        tree.evaluate(p=w.p, theta=w.theta, eps=w.eps, variant=variant, precision=precision, out=out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tree.set_timing(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ph = tree.phase_times()
    tree.set_timing(False)
    return dt, ph


def run_headline(w, pos, mass, args):
    import torch

    from paper_2107_07166_amd import api

    dev = torch.device("cuda:0")
    pd = torch.from_numpy(pos).to(dev)
    md = torch.from_numpy(mass).to(dev)
    ctx = api.Context(0)
    tree = api.Tree(ctx, pd, md, n_leaf=args.n_leaf)
    out = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
    res = {}
    res["t_cons"], res["phases_cons"] = _timed_steps(tree, pd, md, out, w, "conserving", "mixed32",
                                                     args.steps, args.warmup)
    res["force"] = out.cpu().numpy()
    res["t_std"], res["phases_std"] = _timed_steps(tree, pd, md, out, w, "standard", "mixed32",
                                                   args.steps, args.warmup)
    res["force_std"] = out.cpu().numpy()
    res["t_fp64"], res["phases_fp64"] = _timed_steps(tree, pd, md, out, w, "conserving", "fp64",
                                                     max(3, args.steps // 4), 1)
    res["info"] = tree.info()
    d = ctx.diagnostics(pd, md, torch.from_numpy(res["force"]).to(dev))
    ds = ctx.diagnostics(pd, md, torch.from_numpy(res["force_std"]).to(dev))
    res["torque_cons"] = float(d[19])
    res["torque_std"] = float(ds[19])
    res["netforce_cons"] = float(d[18])
    res["netforce_std"] = float(ds[18])
    res["gpu_name"] = torch.cuda.get_device_name(0)
    tree.close()
    ctx.close()
    return res


def run_disk(args):
    """Exponential disk, N = 2^22, p = 6, theta = 0.8: both variants timed the
    same way on one tree; the cost of realignment at a high order and a wide
    angle.  Leaves of up to 128 particles (the conserving variant's fastest
    leaf size here; the far field dominates at p = 6); the standard variant
    is also timed at its own fastest leaf size, 96."""
    import torch

    from paper_2107_07166_amd import api
    from paper_2107_07166_amd.generators import WORKLOADS

    w = WORKLOADS["disk4m"]
    pos, mass = w.make()
    dev = torch.device("cuda:0")
    pd = torch.from_numpy(pos).to(dev)
    md = torch.from_numpy(mass).to(dev)
    ctx = api.Context(0)
    tree = api.Tree(ctx, pd, md, n_leaf=args.disk_n_leaf)
    out = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
    res = {"workload": f"disk4m: exponential disk N={w.n}, scale length 1, sech^2 height 0.05, eps=1e-3, "
                       f"p={w.p}, theta={w.theta}", "n": w.n, "n_leaf": args.disk_n_leaf}
    for variant in ("standard", "conserving"):
        dt, ph = _timed_steps(tree, pd, md, out, w, variant, "mixed32", args.disk_steps, 2)
        d = ctx.diagnostics(pd, md, out)
        res[variant] = {"ms_per_step": dt * 1e3, "evals_per_s": w.n / dt, "phases_ms": ph,
                        "net_torque_rel": float(d[19]), "net_force_rel": float(d[18])}
    res["conserving_overhead"] = res["conserving"]["ms_per_step"] / res["standard"]["ms_per_step"] - 1.0
    res["conserving_overhead_evaluation"] = (res["conserving"]["phases_ms"]["total"]
                                             / res["standard"]["phases_ms"]["total"] - 1.0)
    res["tree"] = tree.info()
    tree.close()
    tree = api.Tree(ctx, pd, md, n_leaf=96)
    dt, ph = _timed_steps(tree, pd, md, out, w, "standard", "mixed32", args.disk_steps, 2)
    res["standard_leaf96"] = {"n_leaf": 96, "ms_per_step": dt * 1e3, "evals_per_s": w.n / dt}
    res["conserving_overhead_vs_fastest_standard"] = res["conserving"]["ms_per_step"] / (dt * 1e3) - 1.0
    tree.close()
    ctx.close()
    return res


def run_serving(args):
    """A bounded serving run on one trace: capacity (every solve queued at
    once) and latency at a fixed Poisson rate for three servers: FP64 one
    solve at a time, mixed precision on several slots with one request per
    launch set, and the same slots solving the small requests of equal order
    and variant together as forests; resident sessions step beside the
    solves."""
    from paper_2107_07166_amd.serve import (Server, close_sessions, make_inputs, make_sessions, make_trace,
                                            summarize)

    trace = make_trace(args.serve_requests, rate=args.serve_rate)
    inputs = {r.rid: make_inputs(r) for r in trace}
    # capacity: the trace's solves four times over, all queued at once (the
    # copies share their inputs); a longer burst averages out the batching
    # decisions that make single 64-solve bursts vary
    copies = 4
    nt = len(trace)
    burst = [dataclasses.replace(r, rid=r.rid + k * nt, arrival=0.0) for k in range(copies) for r in trace]
    burst_inputs = {r.rid + k * nt: inputs[r.rid] for k in range(copies) for r in trace}
    servers = (("fp64_one_at_a_time", "fp64", 1, 1), ("mixed32_slots", "mixed32", args.serve_slots, 1),
               ("mixed32_forests", "mixed32", args.serve_slots, 256))
    res = {"requests": len(trace), "capacity_burst": len(burst), "sessions": args.serve_sessions,
           "rate_per_s": args.serve_rate,
           "slots_batched": args.serve_slots,
           "trace": "Poisson arrivals; N log-uniform in [1e3, 5e5]; ball/Plummer/disk; p in {2,4,6}; "
                    "theta in {0.4,0.6,0.8}; standard/conserving; eps=1e-3"}
    samples = {}
    for name, prec, k, sets in servers:
        srv = Server(slots=k, precision=prec, batch_max_sets=sets)
        sessions = make_sessions(args.serve_sessions, precision=prec, n_max=5e4)
        try:
            # untimed pass first: the first launch of every kernel loads its
            # code and the slots grow their buffers (a running server's state)
            srv.run(burst, inputs=burst_inputs)
            caps = []
            for _ in range(5):  # the median of five bursts
                recs = srv.run(burst, inputs=burst_inputs)
                caps.append(summarize(recs))
            cap = {"solves_per_s": float(np.median([c["solves_per_s"] for c in caps])),
                   "errors": sum(c["errors"] for c in caps)}
            burst_batch = float(np.mean([r.batch for r in recs if r.kind == "solve"]))
            # the latency trace three times: one 64-request p99 is close to the
            # slowest request, and a stall of the host now and then moves it
            reps = []
            for _ in range(args.serve_reps):
                recs = srv.run(trace, sessions=sessions, inputs=inputs)
                reps.append(summarize(recs))
        finally:
            close_sessions(sessions)
            srv.close()
        med = {key: float(np.median([r[key] for r in reps])) for key in ("solves_per_s", "p50_ms", "p99_ms")}
        res[name] = {"slots": k, "capacity_solves_per_s": cap["solves_per_s"],
                     "capacity_each_run": [c["solves_per_s"] for c in caps],
                     "capacity_mean_requests_per_launch_set": burst_batch, "solves_per_s": med["solves_per_s"],
                     "p50_ms": med["p50_ms"], "p99_ms": med["p99_ms"],
                     "p99_ms_each_run": [r["p99_ms"] for r in reps],
                     "session_steps": int(np.median([r["session_steps"] for r in reps])),
                     "step_p50_ms": reps[-1].get("step_p50_ms"), "step_p99_ms": reps[-1].get("step_p99_ms"),
                     "errors": sum(r["errors"] for r in reps) + cap["errors"], "slot_retries": srv.retries}
        samples[name] = {r.rid: r.sample for r in recs if r.kind == "solve" and not r.error}
    a, b = samples["mixed32_forests"], samples["fp64_one_at_a_time"]
    errs = [_erms(a[i], b[i]) for i in a if i in b]
    res["mixed_vs_fp64_rms_per_request"] = {"max": max(errs), "median": float(np.median(errs))}
    res["capacity_ratio"] = (res["mixed32_forests"]["capacity_solves_per_s"]
                             / res["fp64_one_at_a_time"]["capacity_solves_per_s"])
    res["forest_capacity_gain"] = (res["mixed32_forests"]["capacity_solves_per_s"]
                                   / res["mixed32_slots"]["capacity_solves_per_s"])
    return res


def run_distance_test():
    """Two irregular bodies of 4000 particles at distances 3.6 / 8 / 16 (their
    radius is 1), each one leaf, theta = 0.99 (one far pair), eps = 0, FP64:
    rms relative error of the inter-body force for orders 0 and 1 with and
    without realignment.  The exact force is the library's theta = 0
    evaluation (exact pair sums; checked against the oracle's direct sum in
    the GPU tests)."""
    from paper_2107_07166_amd.studies import study_shapes
    r = study_shapes(4000, (3.6, 8.0, 16.0), 5)
    return {"rows": [{k: (v["err"] if isinstance(v, dict) else v) for k, v in row.items()} for row in r["rows"]],
            "net_torque_rel_max": {lab: max(row[lab]["net_torque_rel"] for row in r["rows"])
                                   for lab in r["rows"][0] if isinstance(r["rows"][0][lab], dict)}}


def cpu_baseline(w, pos, mass, budget_s, n_leaf):
    import oracle

    threads = oracle.set_threads(0)
    t0 = time.perf_counter()
    ot = oracle.Tree(pos, mass, n_leaf=n_leaf, theta=w.theta)
    t_tree = time.perf_counter() - t0
    rng = np.random.default_rng(12345)
    probe = rng.choice(w.n, 64, replace=False)
    # the first call also builds the oracle's lazy per-node lists: time a second one
    ot.forces(w.p, w.eps, "conserving", targets=probe[:8])
    t0 = time.perf_counter()
    ot.forces(w.p, w.eps, "conserving", targets=probe)
    t_probe = time.perf_counter() - t0
    k = int(np.clip(64 * budget_s / max(t_probe, 1e-3), 64, 50000))
    sample = rng.choice(w.n, k, replace=False)
    t0 = time.perf_counter()
    f_cons = ot.forces(w.p, w.eps, "conserving", targets=sample)
    t_forces = time.perf_counter() - t0
    f_std = ot.forces(w.p, w.eps, "standard", targets=sample)
    # evaluations/s of the oracle: sampled particles over their share of the tree
    # build plus their force time
    t_per = t_forces / k + t_tree / w.n
    return {"value": 1.0 / t_per, "unit": "particle force evals/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{k} random particles of the N=2^20 Plummer set, conserving p=4 theta=0.5; "
                      f"oracle tree build {t_tree:.2f} s amortised per particle, forces {t_forces:.2f} s"}, \
        sample, f_cons, f_std


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-leaf", type=int, default=64)
    ap.add_argument("--cpu-budget", type=float, default=18.0, help="seconds of oracle force time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--disk-steps", type=int, default=8)
    ap.add_argument("--disk-n-leaf", type=int, default=128)
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-sessions", type=int, default=4)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-rate", type=float, default=100.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-reps", type=int, default=3, help="runs of the latency trace per server (medians)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "is a design, not built", file=sys.stderr)
        sys.exit(2)

    from paper_2107_07166_amd.generators import WORKLOADS

    w = WORKLOADS["plummer1m"]
    pos, mass = w.make()
    g = run_headline(w, pos, mass, args)
    print(f"# headline done: {g['t_cons'] * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    t = g["t_cons"]
    info = g["info"]
    n_int = info["near_interactions"]
    ph = g["phases_cons"]
    p2p_ms = ph["p2p"]
    achieved = P2P_FLOP_PER_PAIR * n_int / (p2p_ms * 1e-3) / 1e12
    m2l_flop = _m2l_pair_flops(w.p, "conserving") * info["far_directed"]
    inter_tflops = (P2P_FLOP_PER_PAIR * n_int + m2l_flop) / (ph["interaction"] * 1e-3) / 1e12
    m2l_flop_std = _m2l_pair_flops(w.p, "standard") * info["far_directed"]
    inter_tflops_std = ((P2P_FLOP_PER_PAIR * n_int + m2l_flop_std)
                        / (g["phases_std"]["interaction"] * 1e-3) / 1e12)
    line = {
        "metric": "particle force evals/s at N=1M p=4 theta=0.5 (conserving variant, end to end)",
        "value": w.n / t,
        "unit": "particle force evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (P2P, M2L) + f64 (tree, moments, L2L, L2P, reductions)",
        "data": "synthetic",
        "config": {"workload": "plummer1m: Plummer sphere N=2^20, a=1, M=1, eps=1e-3, p=4, theta=0.5",
                   "variant": "conserving", "precision": "mixed32", "n_leaf": args.n_leaf},
        "roofline": {"kernel": "p2p_kernel<float>", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "peak_without_packed_fp32": PEAK_FP32_NOPK_TFLOPS,
                     "flop_per_unit": P2P_FLOP_PER_PAIR, "units_per_launch": n_int,
                     "avg_launch_ms": p2p_ms, "traffic": _p2p_traffic()},
        "interaction_pass": {"what": "P2P + M2L algorithmic FLOPs over the window from the first start to "
                                     "the last end of the two (they run side by side)",
                             "p2p_flop": P2P_FLOP_PER_PAIR * n_int,
                             "m2l_flop_per_directed_pair": _m2l_pair_flops(w.p, "conserving"),
                             "m2l_flop": m2l_flop, "window_ms": ph["interaction"],
                             "achieved_tflops": inter_tflops, "frac_of_peak": inter_tflops / PEAK_FP32_TFLOPS,
                             "standard_variant_tflops": inter_tflops_std},
        "standard_variant": {"value": w.n / g["t_std"], "ms_per_step": g["t_std"] * 1e3,
                             "phases_ms": g["phases_std"]},
        "conserving_overhead": g["t_cons"] / g["t_std"] - 1.0,
        "fp64_path": {"value": w.n / g["t_fp64"], "ms_per_step": g["t_fp64"] * 1e3,
                      "phases_ms": g["phases_fp64"]},
        "phases_ms": ph,
        "tree": info,
        "net_torque_rel": {"conserving": g["torque_cons"], "standard": g["torque_std"]},
        "net_force_rel": {"conserving": g["netforce_cons"], "standard": g["netforce_std"]},
        "gpu": g["gpu_name"],
    }
    if not args.no_extra:
        line["disk"] = run_disk(args)
        print(f"# disk done: overhead {line['disk']['conserving_overhead']:.3f}", file=sys.stderr, flush=True)
        line["serving"] = run_serving(args)
        print("# serving done", file=sys.stderr, flush=True)
        line["distance_test"] = run_distance_test()
    if not args.no_cpu:
        cb, sample, f_cons, f_std = cpu_baseline(w, pos, mass, args.cpu_budget, args.n_leaf)
        line["cpu_baseline"] = cb
        line["err_vs_oracle_rms"] = {"conserving": _erms(g["force"][sample], f_cons),
                                     "standard": _erms(g["force_std"][sample], f_std),
                                     "sample": len(sample)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
