"""Continuous-batching server for boosted-frame PIC runs on one GPU.

Requests (2D3V boosted-frame runs of different grids, particle counts,
gamma_boost and step counts) arrive over time.  A request is admitted as soon
as it has arrived and its state fits in the device-memory budget
(pic_state_bytes), first come first served.  All admitted runs stay resident
and are advanced together: every iteration enqueues one batched chunk of
steps in which the tiles of all runs share the same kernel launches (one HIP
graph per step, replayed).  Runs leave the batch when their steps are done,
freeing budget for waiting requests.  Latency = completion - arrival.

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

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class GpuExecutor:
    """Runs requests with libpic on one GPU.  All runs live on one stream:
    pic_step_batch enqueues their batched steps there."""

    def __init__(self, precision: str = "fp32", keep_results: bool = False):
        import torch

        from . import pic

        self.pic = pic
        self.precision = precision
        self.keep = keep_results
        self.stream = torch.cuda.Stream()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def bytes_for(self, req: Request) -> int:
        return self.pic.pic_state_bytes(self.pic.make_params(req.cfg, self.precision))

    def admit(self, req: Request):
        # initialisation (laser transform, plasma creation, first sort) runs
        # on the shared stream and has completed when this returns
        return self.pic.Run(req.cfg, self.precision, stream=self.stream)

    def advance(self, runs, nsteps):
        self.pic.pic_step_batch([r.handle for r in runs], nsteps)

    def wait(self):
        self.stream.synchronize()

    def release(self, run):
        res = run.diag(self.pic.PIC_DIAG_FIELDS | self.pic.PIC_DIAG_PARTICLES) if self.keep else None
        run.close()
        return res


def percentile(xs, q):
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = (len(s) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def schedule(requests, executor, budget_bytes: int, chunk_steps: int = 25, max_batch: int = 256):
    """Run all requests; returns (list of Done, stats dict)."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    waiting = collections.deque()
    active = []  # [req, run, remaining, bytes, admitted]
    done = []
    used = 0
    peak_used = 0
    max_conc = 0
    t_first = None
    while pending or waiting or active:
        now = executor.now()
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        # admission: FIFO, by memory budget
        while waiting and len(active) < max_batch:
            req = waiting[0]
            need = executor.bytes_for(req)
            if need > budget_bytes:
                raise ValueError(f"request {req.rid} needs {need} bytes, over the whole budget")
            if used + need > budget_bytes:
                break
            waiting.popleft()
            run = executor.admit(req)
            used += need
            peak_used = max(peak_used, used)
            active.append([req, run, req.steps, need, executor.now()])
        max_conc = max(max_conc, len(active))
        if not active:
            if pending:
                executor.sleep_until(pending[0].arrival) if hasattr(executor, "sleep_until") else \
                    time.sleep(max(0.0, min(pending[0].arrival - executor.now(), 0.01)))
            continue
        if t_first is None:
            t_first = executor.now()
        nsteps = [min(chunk_steps, a[2]) for a in active]
        executor.advance([a[1] for a in active], nsteps)
        executor.wait()
        t = executor.now()
        keep = []
        for a, n in zip(active, nsteps):
            a[2] -= n
            if a[2] == 0:
                res = executor.release(a[1])
                used -= a[3]
                req = a[0]
                done.append(Done(req.rid, req.arrival, a[4], t, req.particles * req.steps, res))
            else:
                keep.append(a)
        active = keep
    lat = [d.latency for d in done]
    total_ps = sum(d.particle_steps for d in done)
    span = (max(d.finished for d in done) - min(r.arrival for r in requests)) if done else 0.0
    arr = [r.arrival for r in requests]
    arr_span = max(arr) - min(arr) if len(arr) > 1 else float("nan")
    stats = {
        "n_requests": len(done),
        "p50_ms": 1e3 * percentile(lat, 50),
        "p99_ms": 1e3 * percentile(lat, 99),
        "mean_ms": 1e3 * (sum(lat) / len(lat)) if lat else float("nan"),
        "throughput": total_ps / span if span > 0 else float("nan"),
        "offered_load": total_ps / arr_span if arr_span and arr_span > 0 else float("nan"),
        "makespan_s": span,
        "max_concurrency": max_conc,
        "peak_bytes": peak_used,
        "budget_bytes": budget_bytes,
        "chunk_steps": chunk_steps,
    }
    return done, stats


def serve_stream(stream, budget_bytes: int, chunk_steps: int = 25, precision: str = "fp32",
                 keep_results: bool = False):
    """Serve a workloads.serving_stream() list of (arrival_s, cfg) on the GPU."""
    reqs = [Request(i, float(t), c, int(c["steps"])) for i, (t, c) in enumerate(stream)]
    ex = GpuExecutor(precision, keep_results)
    # warm the library, the allocator and the graph capture with one tiny run
    warm = Request(-1, 0.0, dict(reqs[0].cfg, nz=32, nx=32, ppc=1, steps=2), 2)
    r = ex.admit(warm)
    ex.advance([r], [2])
    ex.wait()
    ex.release(r)
    ex.t0 = time.perf_counter()
    done, stats = schedule(reqs, ex, budget_bytes, chunk_steps)
    if keep_results:
        stats["results"] = {d.rid: d.result for d in done}
    return stats
