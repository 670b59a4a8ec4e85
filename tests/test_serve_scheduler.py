"""Host-only tests of the serving scheduler with a fake executor and a
virtual clock: admission by memory budget, first-come-first-served order,
continuous batching (requests join while others run), chunks queued ahead of
the device, rejection of an over-budget request and failure of one run
without disturbing the others, and the latency percentiles."""
import math

import pytest

from paper_0909_5603_amd import serve, workloads


class Chunk:
    def __init__(self, done_at):
        self.done_at = done_at


class FakeExecutor:
    """Virtual clock and a virtual device that runs the queued chunks one
    after the other; a chunk costs a fixed overhead plus time proportional to
    the particle-steps it advances."""

    def __init__(self, ns_per_particle_step=1.0, overhead=1e-4, fail_release=(), fail_admit=()):
        self.t = 0.0
        self.rate = ns_per_particle_step * 1e-9
        self.overhead = overhead
        self.device_free = 0.0
        self.live = {}
        self.log = []
        self.next = 0
        self.fail_release = set(fail_release)
        self.fail_admit = set(fail_admit)
        self.max_queued = 0
        self.queued = []

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)

    def bytes_for(self, req):
        return req.particles * 32 + 1000

    def admit(self, req):
        if req.rid in self.fail_admit:
            raise serve.RunFailed("init failed")
        self.next += 1
        self.live[self.next] = req
        self.log.append(("admit", req.rid, self.t))
        return self.next

    def advance(self, runs, nsteps):
        ps = sum(self.live[r].particles * n for r, n in zip(runs, nsteps))
        self.log.append(("advance", tuple(self.live[r].rid for r in runs), self.t))
        start = max(self.device_free, self.t)
        self.device_free = start + self.overhead + ps * self.rate
        c = Chunk(self.device_free)
        self.queued = [q for q in self.queued if q.done_at > self.t] + [c]
        self.max_queued = max(self.max_queued, len(self.queued))
        return c

    def wait_until(self, chunk, t_limit):
        if chunk.done_at <= t_limit:
            self.t = max(self.t, chunk.done_at)
            return True
        self.t = max(self.t, t_limit)
        return False

    def release(self, run):
        req = self.live.pop(run)
        self.log.append(("release", req.rid, self.t))
        if req.rid in self.fail_release:
            raise serve.RunFailed("device error word set")
        return {"rid": req.rid}


def _reqs(n, seed=5):
    return [serve.Request(i, t, c, c["steps"]) for i, (t, c) in
            enumerate(workloads.serving_stream(n, seed=seed))]


def test_all_requests_complete_and_budget_respected():
    reqs = _reqs(60)
    ex = FakeExecutor()
    budget = 3 * max(ex.bytes_for(r) for r in reqs)
    done, st = serve.schedule(reqs, ex, budget, chunk_steps=50)
    assert sorted(d.rid for d in done) == list(range(60))
    assert st["peak_bytes"] <= budget
    assert st["n_requests"] == 60 and st["n_rejected"] == 0 and st["n_failed"] == 0
    for d in done:
        assert d.finished >= d.admitted >= d.arrival
    # replay the log: resident bytes never exceed the budget
    used = 0
    by = {r.rid: ex.bytes_for(r) for r in reqs}
    for ev, rid, _ in ex.log:
        if ev == "admit":
            used += by[rid]
            assert used <= budget
        elif ev == "release":
            used -= by[rid]


def test_continuous_batching_admits_while_others_run():
    reqs = _reqs(30)
    ex = FakeExecutor(ns_per_particle_step=5.0)
    done, st = serve.schedule(reqs, ex, budget_bytes=1 << 40, chunk_steps=25)
    batches = [rids for ev, rids, _ in ex.log if ev == "advance"]
    # some batch holds several runs, and membership changes over time
    assert max(len(b) for b in batches) > 1
    assert len(set(batches)) > 3
    # a request that arrives while others are active joins before they finish
    first_admit = {rid: t for ev, rid, t in ex.log if ev == "admit"}
    release = {rid: t for ev, rid, t in ex.log if ev == "release"}
    assert any(first_admit[b] < release[a] and first_admit[b] > first_admit[a]
               for a in release for b in release if a != b)
    assert st["max_concurrency"] > 1


def test_next_chunk_is_queued_while_one_runs():
    """The host enqueues the following chunk before the running one ends, so
    the device goes from one chunk to the next without waiting for the host."""
    reqs = _reqs(20)
    ex = FakeExecutor(ns_per_particle_step=5.0)
    done, st = serve.schedule(reqs, ex, budget_bytes=1 << 40, chunk_steps=25, depth=2)
    assert ex.max_queued == 2
    assert st["chunks_queued"] == 2


def test_fifo_admission_under_tight_budget():
    reqs = _reqs(25)
    ex = FakeExecutor()
    budget = max(ex.bytes_for(r) for r in reqs)  # one large run at a time at most
    done, st = serve.schedule(reqs, ex, budget, chunk_steps=100)
    admits = [rid for ev, rid, _ in ex.log if ev == "admit"]
    assert admits == sorted(admits)


def test_request_over_budget_is_rejected_alone():
    reqs = _reqs(12)
    ex = FakeExecutor()
    sizes = sorted(ex.bytes_for(r) for r in reqs)
    budget = sizes[-2]  # the largest request does not fit the whole budget
    big = max(reqs, key=ex.bytes_for).rid
    done, st = serve.schedule(reqs, ex, budget, chunk_steps=50)
    status = {d.rid: d.status for d in done}
    assert status[big] == "rejected"
    assert all(s == "ok" for rid, s in status.items() if rid != big)
    assert st["n_rejected"] == 1 and st["n_requests"] == 11
    assert big not in [rid for ev, rid, _ in ex.log if ev == "admit"]


def test_failed_runs_are_reported_alone():
    reqs = _reqs(15)
    ex = FakeExecutor(fail_release={3, 9}, fail_admit={5})
    done, st = serve.schedule(reqs, ex, budget_bytes=1 << 40, chunk_steps=40)
    status = {d.rid: d.status for d in done}
    assert sorted(status) == list(range(15))
    assert {rid for rid, s in status.items() if s == "failed"} == {3, 5, 9}
    assert st["n_failed"] == 3 and st["n_requests"] == 12
    # the other runs ran to the end, also those batched with the failed ones
    ok = [d for d in done if d.status == "ok"]
    assert all(d.particle_steps == next(r for r in reqs if r.rid == d.rid).particles *
               next(r for r in reqs if r.rid == d.rid).steps for d in ok)


def test_percentiles():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == pytest.approx(50.5)
    assert serve.percentile(xs, 99) == pytest.approx(99.01)
    assert serve.percentile([3.0], 99) == 3.0


def test_latency_accounting_single_request():
    cfg = workloads.config("c1", nz=64, nx=32, ppc=2, steps=100)
    req = serve.Request(0, 0.5, cfg, 100)
    ex = FakeExecutor(ns_per_particle_step=10.0, overhead=0.0)
    done, st = serve.schedule([req], ex, 1 << 40, chunk_steps=30)
    # starts at its arrival, runs 100 steps of 4096 particles at 10 ns each
    assert done[0].latency == pytest.approx(100 * 4096 * 10e-9, rel=1e-9)
    assert st["p50_ms"] == pytest.approx(st["p99_ms"])
    assert not math.isnan(st["throughput"])
