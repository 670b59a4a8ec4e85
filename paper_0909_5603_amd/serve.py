"""Continuous-batching server for boosted-frame PIC runs on one GPU.

Requests (2D3V boosted-frame runs of different grids, particle counts,
gamma_boost and step counts) arrive over time.  A request is admitted as soon
as it has arrived and its state fits in the device-memory budget
(pic_state_bytes), first come first served; one whose state exceeds the whole
budget is rejected on its own.  An admitted run is initialised on a stream of
its own while the batch runs.  All admitted runs stay resident and are
advanced together: every batched chunk of steps shares the same kernel
launches (one HIP graph per step, replayed), and the host keeps the next chunk
queued behind the running one, ordered by events, so the device never waits
for the host.  Runs leave the batch when their steps are done; a run whose
device error word is set is reported as failed without disturbing the
others.  Latency = completion - arrival.

The scheduler is written against a small executor interface so that its
bookkeeping can be tested on the CPU with a virtual clock; GpuExecutor is the
production executor over libpic.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after the stream start
    cfg: dict
    steps: int

    @property
    def particles(self) -> int:
        ny = self.cfg.get("ny", 1) if self.cfg["dims"] == 3 else 1
        return int(self.cfg["nz"] * self.cfg["nx"] * ny * self.cfg["ppc"])


@dataclasses.dataclass
class Done:
    rid: int
    arrival: float
    admitted: float
    finished: float
    particle_steps: int
    result: dict | None = None
    status: str = "ok"  # "ok", "rejected" (over the whole budget) or "failed"
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class RunFailed(RuntimeError):
    """A run ended with its device error word set (or could not start)."""


class _Slot:
    """A resident run, its own stream and the event its last work was
    ordered behind (its initialisation, then the last chunk it took part in)."""

    __slots__ = ("run", "stream", "pending")

    def __init__(self, run, stream, pending):
        self.run, self.stream, self.pending = run, stream, pending


class GpuExecutor:
    """Runs requests with libpic on one GPU.

    Every run owns a stream (from a pool) on which it is initialised and its
    results are read.  pic_step_batch enqueues a chunk on the first run's
    stream; the chunk waits on the previous chunk and on each member's
    pending work (events), and the members' streams then wait on the chunk's
    event, so reading a finished run's results waits only for the chunks it
    took part in, never for the chunk queued behind them."""

    def __init__(self, precision: str = "fp32", keep_results: bool = False, n_streams: int = 32):
        import torch

        from . import pic

        self.torch = torch
        self.pic = pic
        self.precision = precision
        self.keep = keep_results
        self.pool = [torch.cuda.Stream() for _ in range(n_streams)]
        self.last_chunk = None
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        dt = t - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.01))

    def bytes_for(self, req: Request) -> int:
        return self.pic.pic_state_bytes(self.pic.make_params(req.cfg, self.precision))

    def admit(self, req: Request):
        s = self.pool.pop() if self.pool else self.torch.cuda.Stream()
        try:
            run = self.pic.Run(req.cfg, self.precision, stream=s)
        except self.pic.PicError as e:
            self.pool.append(s)
            raise RunFailed(str(e)) from e
        ev = self.torch.cuda.Event()
        ev.record(s)
        return _Slot(run, s, ev)

    def advance(self, slots, nsteps):
        bs = slots[0].stream
        if self.last_chunk is not None:
            bs.wait_event(self.last_chunk)
        for sl in slots:
            if sl.pending is not None and sl.stream is not bs:
                bs.wait_event(sl.pending)
        self.pic.pic_step_batch([sl.run.handle for sl in slots], nsteps)
        ev = self.torch.cuda.Event()
        ev.record(bs)
        for sl, n in zip(slots, nsteps):
            if n > 0:
                if sl.stream is not bs:
                    sl.stream.wait_event(ev)
                sl.pending = ev
        self.last_chunk = ev
        return ev

    def wait_until(self, token, t_limit: float) -> bool:
        """True once the chunk has run; False if t_limit passes first."""
        while not token.query():
            if self.now() >= t_limit:
                return False
            time.sleep(5e-5)
        return True

    def release(self, slot):
        pic = self.pic
        try:
            what = pic.PIC_DIAG_FIELDS | pic.PIC_DIAG_PARTICLES if self.keep else 0
            res = slot.run.diag(what)  # raises on a set device error word
            if self.keep:
                p = slot.run.particles()
                res = dict(res, particles={k: p[k] for k in ("id", "ux", "uy", "uz")})
            return res if self.keep else None
        except pic.PicError as e:
            raise RunFailed(str(e)) from e
        finally:
            slot.run.close()
            self.pool.append(slot.stream)


def percentile(xs, q):
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = (len(s) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def schedule(requests, executor, budget_bytes: int, chunk_steps: int = 25, max_batch: int = 256,
             depth: int = 2):
    """Run all requests; returns (list of Done, stats dict).  depth = chunks
    kept queued on the device."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    waiting = collections.deque()
    active = []  # dicts: req, slot, unq (steps not yet enqueued), left (not yet run), bytes, admitted
    inflight = collections.deque()  # (token, [(entry, nsteps)])
    done = []
    used = 0
    peak_used = 0
    max_conc = 0

    def finish(entry, t):
        nonlocal used
        req = entry["req"]
        try:
            res = executor.release(entry["slot"])
            done.append(Done(req.rid, req.arrival, entry["admitted"], t, req.particles * req.steps, res))
        except RunFailed as e:
            done.append(Done(req.rid, req.arrival, entry["admitted"], t, 0, None, "failed", str(e)))
        used -= entry["bytes"]

    while pending or waiting or active:
        now = executor.now()
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        # admission: FIFO, by memory budget; a request larger than the whole
        # budget is rejected alone
        while waiting and len(active) < max_batch:
            req = waiting[0]
            need = executor.bytes_for(req)
            if need > budget_bytes:
                waiting.popleft()
                done.append(Done(req.rid, req.arrival, now, now, 0, None, "rejected",
                                 f"needs {need} bytes, over the budget of {budget_bytes}"))
                continue
            if used + need > budget_bytes:
                break
            waiting.popleft()
            try:
                slot = executor.admit(req)
            except RunFailed as e:
                t = executor.now()
                done.append(Done(req.rid, req.arrival, t, t, 0, None, "failed", str(e)))
                continue
            used += need
            peak_used = max(peak_used, used)
            active.append({"req": req, "slot": slot, "unq": req.steps, "left": req.steps,
                           "bytes": need, "admitted": executor.now()})
        max_conc = max(max_conc, len(active))
        # keep `depth` chunks queued on the device
        members = [a for a in active if a["unq"] > 0]
        if members and len(inflight) < depth:
            nsteps = [min(chunk_steps, a["unq"]) for a in members]
            token = executor.advance([a["slot"] for a in members], nsteps)
            for a, n in zip(members, nsteps):
                a["unq"] -= n
            inflight.append((token, list(zip(members, nsteps))))
            continue
        if inflight:
            token, parts = inflight[0]
            # wake up for the chunk's end or the next arrival, whichever is first
            t_next = pending[0].arrival if pending else math.inf
            if waiting:  # blocked by the budget: only a finishing run helps
                t_next = math.inf
            if not executor.wait_until(token, t_next):
                continue
            inflight.popleft()
            t = executor.now()
            for a, n in parts:
                a["left"] -= n
                if a["left"] == 0:
                    finish(a, t)
            active = [a for a in active if a["left"] > 0]
            continue
        if pending and not active:
            executor.sleep_until(pending[0].arrival)
    ok = [d for d in done if d.status == "ok"]
    lat = [d.latency for d in ok]
    total_ps = sum(d.particle_steps for d in ok)
    span = (max(d.finished for d in ok) - min(r.arrival for r in requests)) if ok else 0.0
    arr = [r.arrival for r in requests]
    arr_span = max(arr) - min(arr) if len(arr) > 1 else float("nan")
    offered = sum(r.particles * r.steps for r in requests)
    stats = {
        "n_requests": len(ok),
        "n_rejected": sum(d.status == "rejected" for d in done),
        "n_failed": sum(d.status == "failed" for d in done),
        "p50_ms": 1e3 * percentile(lat, 50),
        "p99_ms": 1e3 * percentile(lat, 99),
        "mean_ms": 1e3 * (sum(lat) / len(lat)) if lat else float("nan"),
        "throughput": total_ps / span if span > 0 else float("nan"),
        "offered_load": offered / arr_span if arr_span and arr_span > 0 else float("nan"),
        "makespan_s": span,
        "arrival_span_s": arr_span,
        "max_concurrency": max_conc,
        "peak_bytes": peak_used,
        "budget_bytes": budget_bytes,
        "chunk_steps": chunk_steps,
        "chunks_queued": depth,
    }
    return done, stats


def serve_stream(stream, budget_bytes: int, chunk_steps: int = 25, precision: str = "fp32",
                 keep_results: bool = False, depth: int = 2):
    """Serve a workloads.serving_stream() list of (arrival_s, cfg) on the GPU."""
    reqs = [Request(i, float(t), c, int(c["steps"])) for i, (t, c) in enumerate(stream)]
    ex = GpuExecutor(precision, keep_results)
    # warm the library, the allocator and the graph capture with one tiny run
    warm = Request(-1, 0.0, dict(reqs[0].cfg, nz=32, nx=32, ppc=1, steps=2), 2)
    s = ex.admit(warm)
    tok = ex.advance([s], [2])
    ex.wait_until(tok, math.inf)
    ex.release(s)
    ex.last_chunk = None
    ex.t0 = time.perf_counter()
    done, stats = schedule(reqs, ex, budget_bytes, chunk_steps, depth=depth)
    if keep_results:
        stats["results"] = {d.rid: d.result for d in done if d.status == "ok"}
    stats["status"] = {d.rid: d.status for d in done if d.status != "ok"}
    return stats
