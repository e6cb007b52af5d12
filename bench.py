"""Benchmark: particle force evaluations per second on one MI355X.

Workload: Plummer sphere, N = 2^20 equal masses (total 1), scale radius 1,
softening 1e-3, expansion order p = 4, theta = tan(theta_MAC) = 0.5, seeded
synthetic input resident in HBM.  One step = one full force evaluation of the
conserving (torque-free) variant in the mixed path: tree rebuild (keys, sort,
octree, centres of mass, r_max), walk, moments, M2L, L2L, P2P, L2P.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Besides the headline value it reports the standard
variant and the FP64 path at the same workload, per-phase device times
(HIP events on the library's stream), the roofline of the dominant kernel
(P2P), and the CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
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
P2P_TRAFFIC_BYTES = (2 * 225760 + 32009) * 1024
P2P_TRAFFIC_SOURCE_SHA = "9b57e608a2569034"


def _p2p_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2107_07166_amd", "csrc", "p2p.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return P2P_TRAFFIC_BYTES if sha == P2P_TRAFFIC_SOURCE_SHA else None


def _erms(f, ref):
    return float(np.sqrt(np.mean(((f - ref) ** 2).sum(1) / (ref ** 2).sum(1))))


def run_gpu(w, pos, mass, args):
    import torch

    from paper_2107_07166_amd import api

    dev = torch.device("cuda:0")
    pd = torch.from_numpy(pos).to(dev)
    md = torch.from_numpy(mass).to(dev)
    ctx = api.Context(0)
    tree = api.Tree(ctx, pd, md, n_leaf=args.n_leaf)
    out = torch.empty((w.n, 3), dtype=torch.float64, device=dev)

    def step(variant, precision):
        tree.rebuild(pd, md)
        tree.evaluate(p=w.p, theta=w.theta, eps=w.eps, variant=variant, precision=precision, out=out)

    def timed(variant, precision, steps, warmup, phases=None):
        for _ in range(warmup):
            step(variant, precision)
        torch.cuda.synchronize()
        if phases is not None:
            tree.set_timing(True)   # HIP events around every phase of the timed steps
        t0 = time.perf_counter()
        for _ in range(steps):
            step(variant, precision)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        if phases is not None:
            phases.update(tree.phase_times())   # averages over the timed steps
            tree.set_timing(False)
        return dt

    res = {}
    phases = {}
    res["t_cons"] = timed("conserving", "mixed32", args.steps, args.warmup, phases)
    res["phases_ms"] = phases
    res["t_std"] = timed("standard", "mixed32", max(3, args.steps // 2), 2)
    res["t_fp64"] = timed("conserving", "fp64", max(3, args.steps // 4), 1)
    res["info"] = tree.info()
    step("conserving", "mixed32")
    torch.cuda.synchronize()
    res["force"] = out.cpu().numpy()
    step("standard", "mixed32")
    torch.cuda.synchronize()
    res["force_std"] = out.cpu().numpy()
    d = ctx.diagnostics(pd, md, torch.from_numpy(res["force"]).to(dev))
    ds = ctx.diagnostics(pd, md, torch.from_numpy(res["force_std"]).to(dev))
    res["torque_cons"] = float(d[19])
    res["torque_std"] = float(ds[19])
    res["netforce_cons"] = float(d[18])
    res["gpu_name"] = torch.cuda.get_device_name(0)
    tree.close()
    ctx.close()
    return res


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "is a design, not built", file=sys.stderr)
        sys.exit(2)

    from paper_2107_07166_amd.generators import WORKLOADS

    w = WORKLOADS["plummer1m"]
    pos, mass = w.make()
    g = run_gpu(w, pos, mass, args)
    t = g["t_cons"]
    n_int = g["info"]["near_interactions"]
    p2p_ms = g["phases_ms"]["p2p"]
    achieved = P2P_FLOP_PER_PAIR * n_int / (p2p_ms * 1e-3) / 1e12
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
        "standard_variant": {"value": w.n / g["t_std"], "ms_per_step": g["t_std"] * 1e3},
        "conserving_overhead": g["t_cons"] / g["t_std"] - 1.0,
        "fp64_path": {"value": w.n / g["t_fp64"], "ms_per_step": g["t_fp64"] * 1e3},
        "phases_ms": g["phases_ms"],
        "tree": g["info"],
        "net_torque_rel": {"conserving": g["torque_cons"], "standard": g["torque_std"]},
        "net_force_rel_conserving": g["netforce_cons"],
        "gpu": g["gpu_name"],
    }
    if not args.no_cpu:
        cb, sample, f_cons, f_std = cpu_baseline(w, pos, mass, args.cpu_budget, args.n_leaf)
        line["cpu_baseline"] = cb
        line["err_vs_oracle_rms"] = {"conserving": _erms(g["force"][sample], f_cons),
                                     "standard": _erms(g["force_std"][sample], f_std),
                                     "sample": len(sample)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
