"""Continuous-batching server for gravity solves and resident leapfrog sessions.

Requests arrive over time (a Poisson trace); each asks for the forces on one
particle set (N, p, theta, variant) or for the next leapfrog step of one of
the persistent sessions.  The server keeps `slots` workers busy: as soon as a
worker is free and the solve at the head of the queue fits in the device
memory budget, it is admitted, so requests that arrive while others run start
as slots and memory free up.  The budget counts what the slots really hold:
a slot keeps its grow-only tree, its context's reusable blocks and its
request buffers between solves, and a running solve reserves what the slot
holds plus its footprint (tfmm_footprint_bytes plus the request buffers)
when the budget has room for that, else the larger of the two; the library
part of the reservation is the slot context's budget, so a solve cannot
outgrow it (a reused tree that would, under the smaller reservation, gives
its memory back and solves once more from scratch).  When the head solve does not fit, idle slots give their
memory back, the largest first.  Solves go first; a
session step takes a free worker only while no admissible solve is waiting,
and session steps hold at most `step_slots` workers at once (default half),
so an arriving solve finds a worker ready; while any solve runs, no new
session step starts (`steps_beside_solves`, default 0), since steps would
share the device with the solves and stretch their latency.  Every worker owns a
libtfmm context, its own HIP stream (default priority), one reusable tree
(device buffers are grow-only) and, during a run, one host thread fed
through a queue, so the work of several requests overlaps on the GPU.  Sessions keep particles and tree resident in HBM between steps and
are re-queued after every step.

The slots live as long as the Server (created by the first run, kept with
what they hold for later runs, released by close()).  Every solve is
deterministic, so its result is the same alone and in a mix.  Latency is
arrival -> completion on the device.
"""

from __future__ import annotations

import collections
import itertools
import math
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import _lib, api, generators
from .session import Session, footprint_bytes as session_footprint


@dataclass
class Request:
    rid: int
    arrival: float                # seconds after the start of the trace
    kind: str = "solve"           # "solve" or "step"
    n: int = 0
    gen: str = "plummer"
    seed: int = 0
    p: int = 4
    theta: float = 0.5
    eps: float = 1e-3
    variant: str = "conserving"
    session: int = -1
    dt: float = 1e-3


@dataclass
class Record:
    rid: int
    kind: str
    n: int
    p: int
    theta: float
    variant: str
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    footprint: int = 0
    worker: int = -1
    batch: int = 1                       # requests solved together in one forest
    sample: Optional[np.ndarray] = None  # forces at the first `sample_k` particles
    full: Optional[np.ndarray] = None    # all forces (only when requested)
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_trace(n_requests: int = 512, rate: float = 100.0, seed: int = generators.SEED_BASE + 4,
               n_min: float = 1e3, n_max: float = 5e5, p_choices=(2, 4, 6), theta_choices=(0.4, 0.6, 0.8),
               kinds=("ball", "plummer", "disk"), variants=("standard", "conserving")) -> List[Request]:
    """Poisson arrivals at `rate`/s; N log-uniform in [n_min, n_max]; generator,
    p, theta and variant uniform over the given choices."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    out = []
    for i in range(n_requests):
        n = int(round(10 ** rng.uniform(math.log10(n_min), math.log10(n_max))))
        out.append(Request(rid=i, arrival=float(t[i]), kind="solve", n=n, gen=str(rng.choice(kinds)),
                           seed=int(rng.integers(1 << 30)), p=int(rng.choice(p_choices)),
                           theta=float(rng.choice(theta_choices)), variant=str(rng.choice(variants))))
    return out


def make_inputs(req: Request):
    """Pinned host copies of a request's particle set (the client's payload)."""
    pos, mass = generators.generate(req.gen, req.n, req.seed)
    hp = torch.empty((req.n, 3), dtype=torch.float64, pin_memory=True)
    hm = torch.empty((req.n,), dtype=torch.float64, pin_memory=True)
    hp.copy_(torch.from_numpy(pos))
    hm.copy_(torch.from_numpy(mass))
    return hp, hm


# Device bytes per particle of a worker's request buffers (pos, mass, force).
STATE_BYTES = 56


class _Worker:
    """One slot: a libtfmm context, a stream, a reusable tree and request
    buffers.  Everything it keeps between requests counts as held memory."""

    def __init__(self, wid: int, device: int, n_leaf: int):
        self.wid = wid
        self.ctx = api.Context(device)
        self.stream = torch.cuda.Stream(device=device)
        self.dev = torch.device("cuda", device)
        self.n_leaf = n_leaf
        self.tree: Optional[api.Tree] = None
        self.retries = 0  # solves run again from scratch after outgrowing the reservation
        self.pos = None
        self.mass = None
        self.force = None

    def tensor_bytes(self) -> int:
        return 0 if self.pos is None else STATE_BYTES * int(self.pos.shape[0])

    def held(self) -> int:
        """Device bytes this slot keeps: the context's (trees, scratch, blocks
        kept for reuse) plus the request buffers."""
        return self.ctx.bytes_held() + self.tensor_bytes()

    def shrink(self) -> None:
        """Give everything back (idle slots only)."""
        if self.tree is not None:
            self.tree.close()
            self.tree = None
        self.pos = self.mass = self.force = None
        self.ctx.trim()

    def _buffers(self, n: int):
        if self.pos is None or self.pos.shape[0] < n:
            self.pos = self.mass = self.force = None
            cap = max(n, 1024)
            self.pos = torch.empty((cap, 3), dtype=torch.float64, device=self.dev)
            self.mass = torch.empty((cap,), dtype=torch.float64, device=self.dev)
            self.force = torch.empty((cap, 3), dtype=torch.float64, device=self.dev)
        return self.pos[:n], self.mass[:n], self.force[:n]

    def solve(self, reqs: List[Request], inputs, precision: str):
        """Forces for one request, or for several as one forest (one set of
        launches; every set's forces are those of the request solved alone).
        Returns the force buffer and the request boundaries in it.  A tree
        reused from earlier requests may need to grow past the slot's
        reservation: then the slot gives its memory back and solves once more
        from scratch."""
        off = np.cumsum([0] + [r.n for r in reqs]).astype(np.int64)
        for attempt in (0, 1):
            try:
                return self._solve(reqs, inputs, precision, off), off
            except api.TfmmError as e:
                if attempt or e.status != _lib.ENOMEM or (self.tree is None and self.ctx.bytes_held() == 0):
                    raise
                self.stream.synchronize()
                self.shrink()
                self.retries += 1

    def _solve(self, reqs, inputs, precision, off):
        r0 = reqs[0]
        with torch.cuda.stream(self.stream):
            pos, mass, force = self._buffers(int(off[-1]))
            for r, a, b in zip(reqs, off[:-1], off[1:]):
                hp, hm = inputs[r.rid]
                pos[a:b].copy_(hp, non_blocking=True)
                mass[a:b].copy_(hm, non_blocking=True)
            sets = None if len(reqs) == 1 else off
            if self.tree is None:
                self.tree = api.Tree(self.ctx, pos, mass, n_leaf=self.n_leaf, offsets=sets)
            else:
                self.tree.rebuild(pos, mass, offsets=sets)
            if sets is None:
                self.tree.evaluate(p=r0.p, theta=r0.theta, eps=r0.eps, variant=r0.variant, precision=precision,
                                   out=force)
            else:
                self.tree.evaluate_forest([r.theta for r in reqs], p=r0.p, eps=r0.eps, variant=r0.variant,
                                          precision=precision, out=force)
            self.stream.synchronize()
        return force

    def close(self):
        if self.tree is not None:
            self.tree.close()
        self.ctx.close()


class Server:
    def __init__(self, slots: int = 8, precision: str = "mixed32", budget_bytes: int = 64 << 30,
                 n_leaf: int = 64, device: int = 0, sample_k: int = 16, keep_full: bool = False,
                 step_slots: Optional[int] = None, batch_max_n: int = 200000, batch_max_total: int = 1 << 18,
                 batch_max_sets: int = 256, steps_beside_solves: int = 0):
        """batch_max_n: requests of at most this many particles are solved
        together as one forest (same p, variant and softening; theta may
        differ), up to batch_max_total particles and batch_max_sets requests
        per forest; batch_max_sets = 1 solves every request alone.  Forests
        of a quarter million particles at most keep the slots evenly loaded:
        a forest of a million particles can end a queue of solves long
        after the other slots are idle.  n_leaf 64: forests of the serving
        trace ran at 2.4k solves/s with leaves of 32 particles, 3.2-3.3k with
        64, 3.5k with 96 and 3.2k with 128 (FP64 one at a time: 585, 578-587,
        559, 569)."""
        self._workers = None  # the slots, created at the first run and kept until close()
        self.batch_max_n = int(batch_max_n)
        self.batch_max_total = int(batch_max_total)
        self.batch_max_sets = max(1, min(int(batch_max_sets), 4096))
        self.slots = int(slots)
        # most workers session steps may hold at once (the rest stay ready for solves)
        self.step_slots = max(1, self.slots // 2) if step_slots is None else max(1, int(step_slots))
        # session steps are background work: while a solve runs, at most this
        # many of them may start (they share the device with the solves)
        self.steps_beside_solves = max(0, int(steps_beside_solves))
        self.precision = precision
        self.budget = int(budget_bytes)
        self.n_leaf = int(n_leaf)
        self.device = int(device)
        self.sample_k = int(sample_k)
        self.keep_full = bool(keep_full)

    def footprint(self, req: Request, n: Optional[int] = None) -> int:
        """Device bytes a solve may need: the library's estimate for its tree
        plus its request buffers (n: the particles of a whole forest)."""
        n = req.n if n is None else n
        return api.footprint_bytes(n, req.p, self.n_leaf, self.precision) + STATE_BYTES * max(n, 1024)

    def _batch(self, pending, room: int) -> List[Request]:
        """The head request and the waiting requests that can share its forest
        (queue order), within the batch limits and `room` bytes."""
        head = pending[0]
        batch, tot = [head], head.n
        if self.batch_max_sets == 1 or head.n > self.batch_max_n:
            return batch
        for r in itertools.islice(pending, 1, None):
            if len(batch) >= self.batch_max_sets:
                break
            if (r.n <= self.batch_max_n and (r.p, r.variant, r.eps) == (head.p, head.variant, head.eps)
                    and tot + r.n <= self.batch_max_total and self.footprint(head, tot + r.n) <= room):
                batch.append(r)
                tot += r.n
        return batch

    def run(self, requests: List[Request], sessions: Optional[List[Session]] = None,
            session_dt: float = 1e-3, inputs=None) -> List[Record]:
        """Serve `requests` (sorted by arrival) and keep `sessions` stepping until
        the last request is done.  Returns one record per solve and per session step."""
        requests = sorted(requests, key=lambda r: r.arrival)
        inputs = inputs if inputs is not None else {r.rid: make_inputs(r) for r in requests}
        sessions = sessions or []
        if self._workers is None:
            self._workers = [_Worker(i, self.device, self.n_leaf) for i in range(self.slots)]
        workers = self._workers
        lock = threading.Condition()
        pending = collections.deque()      # solves, FIFO
        steps_q = collections.deque()      # session steps, FIFO
        records: List[Record] = []
        # Memory: the sessions' footprints, plus per slot either the bytes
        # reserved for the solve it runs (what it held plus the solve's
        # footprint, or the larger of the two when the budget is short; the
        # library part enforced through the slot context's budget) or, while
        # it runs no solve, what it holds.
        sess_bytes = sum(session_footprint(s.n, s.params["p"], s.n_leaf, s.params["precision"]) for s in sessions)
        reserved = {}                      # slot -> bytes reserved for its running solve
        state = {"free_workers": list(range(self.slots)), "solves_left": len(requests), "next_step_id": 10**9,
                 "stop": False, "error": None}
        self.peak_reserved = sess_bytes
        self.over_reservation = 0
        if sess_bytes > self.budget:
            raise MemoryError("the resident sessions alone exceed the memory budget")

        def total_bytes(exclude: int = -1) -> int:
            tot = sess_bytes
            for v, w in enumerate(workers):
                if v != exclude:
                    tot += reserved[v] if v in reserved else w.held()
            return tot
        t0 = time.perf_counter()
        for k, s in enumerate(sessions):  # every session starts with one queued step
            steps_q.append(Request(rid=state["next_step_id"] + k, arrival=0.0, kind="step", n=s.n, session=k,
                                   p=s.params["p"], theta=s.params["theta"], variant=s.params["variant"],
                                   dt=session_dt))
        state["next_step_id"] += len(sessions)
        busy_sessions = set()

        def execute(wid: int, reqs: List[Request], admitted: float, fp: int):
            req = reqs[0]
            recs = [Record(r.rid, r.kind, r.n, r.p, r.theta, r.variant, r.arrival, admitted, footprint=fp,
                           worker=wid, batch=len(reqs)) for r in reqs]
            try:
                if req.kind == "solve":
                    f, off = workers[wid].solve(reqs, inputs, self.precision)
                    for rec, a, b in zip(recs, off[:-1], off[1:]):
                        rec.sample = f[a: a + min(self.sample_k, b - a)].cpu().numpy()
                        if self.keep_full:
                            rec.full = f[a:b].cpu().numpy()
                else:
                    s = sessions[req.session]
                    s.step(req.dt, 1)
                    with s._stream_ctx():  # the copy waits for the step on the session's stream
                        recs[0].sample = s.force[: self.sample_k].cpu().numpy()
            except Exception as e:  # recorded, the server keeps going
                for rec in recs:
                    rec.error = repr(e)
            done = time.perf_counter() - t0
            for rec in recs:
                rec.done = done
            rec = recs[0]
            with lock:
                records.extend(recs)
                if req.kind == "solve":
                    held = workers[wid].held()
                    if held > reserved.pop(wid):
                        self.over_reservation += 1
                    state["solves_left"] -= len(reqs)
                else:
                    busy_sessions.discard(req.session)
                    if state["solves_left"] > 0:
                        steps_q.append(Request(rid=state["next_step_id"], arrival=rec.done, kind="step",
                                               n=req.n, session=req.session, p=req.p, theta=req.theta,
                                               variant=req.variant, dt=req.dt))
                        state["next_step_id"] += 1
                state["free_workers"].append(wid)
                lock.notify_all()

        # one thread per slot for the whole run, fed through its own queue
        jobs = [queue.SimpleQueue() for _ in workers]

        def slot_loop(wid: int):
            while True:
                job = jobs[wid].get()
                if job is None:
                    return
                execute(wid, *job)

        threads = [threading.Thread(target=slot_loop, args=(v,), daemon=True) for v in range(len(workers))]
        for th in threads:
            th.start()
        nxt = 0
        with lock:
            while True:
                now = time.perf_counter() - t0
                while nxt < len(requests) and requests[nxt].arrival <= now:
                    pending.append(requests[nxt])
                    nxt += 1
                # admit solves from the head while a worker is free and memory allows (FIFO)
                while pending and state["free_workers"]:
                    req = pending[0]
                    fp = self.footprint(req)
                    if fp > self.budget - sess_bytes:
                        pending.popleft()
                        records.append(Record(req.rid, req.kind, req.n, req.p, req.theta, req.variant, req.arrival,
                                              error="footprint exceeds the budget"))
                        state["solves_left"] -= 1
                        continue
                    batch = self._batch(pending, self.budget - sess_bytes)
                    n_batch = sum(r.n for r in batch)
                    fp = self.footprint(req, n_batch)
                    lib_fp = api.footprint_bytes(n_batch, req.p, self.n_leaf, self.precision)
                    free = state["free_workers"]

                    def need_of(v, roomy=False):
                        # bytes slot v reserves for this solve, for the library and the
                        # buffers: the larger of what it holds and the footprint (tight;
                        # a reused tree that must grow past it solves again from scratch),
                        # or what it holds plus the footprint (roomy: room for every
                        # grow-only buffer to grow)
                        held_lib, held_buf = workers[v].ctx.bytes_held(), workers[v].tensor_bytes()
                        if roomy:
                            lib_need = held_lib + lib_fp
                            return lib_need, lib_need + held_buf + fp - lib_fp
                        lib_need = max(held_lib, lib_fp)
                        return lib_need, lib_need + max(held_buf, fp - lib_fp)

                    # the free slot that grows least (ties: the one holding most)
                    wid = min(free, key=lambda v: (need_of(v)[1] - workers[v].held(), -workers[v].held()))
                    w = workers[wid]
                    lib_need, need = need_of(wid, roomy=True)
                    total = total_bytes(exclude=wid) + need
                    if total > self.budget:
                        lib_need, need = need_of(wid)
                        total = total_bytes(exclude=wid) + need
                    if total > self.budget:
                        # give back what idle slots keep, the largest first, then the chosen
                        # slot's own leftovers (its buffers may exceed what this solve needs)
                        for v in sorted((v for v in free if v != wid), key=lambda v: -workers[v].held()) + [wid]:
                            workers[v].shrink()
                            lib_need, need = need_of(wid)
                            total = total_bytes(exclude=wid) + need
                            if total <= self.budget:
                                break
                    if total > self.budget:
                        break  # wait for running solves: alone, the solve fits (checked above)
                    for r in batch:
                        pending.remove(r)
                    reserved[wid] = need
                    w.ctx.set_budget(lib_need)
                    self.peak_reserved = max(self.peak_reserved, total)
                    free.remove(wid)
                    jobs[wid].put((batch, now, fp))
                # session steps fill the workers no admissible solve is waiting for
                # (here either no solve waits or the head solve does not fit yet)
                rounds = len(steps_q)
                step_cap = self.step_slots if not reserved else min(self.step_slots, self.steps_beside_solves)
                while steps_q and state["free_workers"] and rounds > 0 and len(busy_sessions) < step_cap:
                    rounds -= 1
                    req = steps_q.popleft()
                    if req.session in busy_sessions:
                        steps_q.append(req)
                        continue
                    busy_sessions.add(req.session)
                    wid = state["free_workers"].pop()
                    jobs[wid].put(([req], now, 0))
                if state["solves_left"] <= 0 and len(state["free_workers"]) == self.slots:
                    break
                wait = None
                if nxt < len(requests):
                    wait = max(0.0, requests[nxt].arrival - (time.perf_counter() - t0))
                lock.wait(timeout=wait if wait is not None else 0.05)
        for q in jobs:
            q.put(None)
        for th in threads:
            th.join()
        self.retries = sum(w.retries for w in workers)
        return sorted(records, key=lambda r: (r.kind, r.rid))

    def close(self) -> None:
        """Release the slots (their contexts, trees and buffers)."""
        if self._workers is not None:
            for w in self._workers:
                w.close()
            self._workers = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_sessions(count: int = 16, seed: int = generators.SEED_BASE + 4, n_min: float = 1e3, n_max: float = 5e5,
                  precision: str = "mixed32", n_leaf: int = 32, device: int = 0,
                  p_choices=(2, 4, 6), theta_choices=(0.4, 0.6, 0.8), kinds=("ball", "plummer", "disk"),
                  variants=("standard", "conserving")) -> List[Session]:
    """Persistent leapfrog sessions drawn like the requests; each has its own
    context and stream so that different workers can step them concurrently."""
    rng = np.random.default_rng(seed + 7919)
    out = []
    dev = torch.device("cuda", device)
    for _ in range(count):
        n = int(round(10 ** rng.uniform(math.log10(n_min), math.log10(n_max))))
        kind = str(rng.choice(kinds))
        w = generators.Workload(kind, int(rng.integers(1 << 20)), kind, n, 1, 0.5)
        pos, mass, vel = w.make(velocities=True)
        ctx = api.Context(device)
        s = Session(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev),
                    torch.from_numpy(mass).to(dev), p=int(rng.choice(p_choices)),
                    theta=float(rng.choice(theta_choices)), eps=1e-3, variant=str(rng.choice(variants)),
                    precision=precision, n_leaf=n_leaf, stream=torch.cuda.Stream(device=device))
        s._owned_ctx = ctx
        out.append(s)
    return out


def close_sessions(sessions: List[Session]) -> None:
    for s in sessions:
        s.close()
        ctx = getattr(s, "_owned_ctx", None)
        if ctx is not None:
            ctx.close()


def summarize(records: List[Record]) -> dict:
    solves = [r for r in records if r.kind == "solve" and not r.error]
    steps = [r for r in records if r.kind == "step" and not r.error]
    out = {"solves": len(solves), "session_steps": len(steps),
           "errors": sum(1 for r in records if r.error)}
    if solves:
        lat = np.array([r.latency for r in solves])
        t_first = min(r.arrival for r in solves)
        t_last = max(r.done for r in solves)
        out.update(solves_per_s=len(solves) / (t_last - t_first), p50_ms=float(np.percentile(lat, 50) * 1e3),
                   p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                   particles_per_s=float(sum(r.n for r in solves) / (t_last - t_first)))
    if steps:
        lat = np.array([r.done - r.admitted for r in steps])
        out.update(step_p50_ms=float(np.percentile(lat, 50) * 1e3), step_p99_ms=float(np.percentile(lat, 99) * 1e3))
    return out
