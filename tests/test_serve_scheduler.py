"""Host-only tests of the serving scheduler with a fake executor and a
virtual clock: admission by memory budget, first-come-first-served order,
continuous batching (requests join while others run), slot reuse and the
latency percentiles."""
import pytest

from paper_0909_5603_amd import serve, workloads


class FakeExecutor:
    """Virtual clock; a batched chunk costs a fixed overhead plus time
    proportional to the particle-steps it advances."""

    def __init__(self, ns_per_particle_step=1.0, overhead=1e-4):
        self.t = 0.0
        self.rate = ns_per_particle_step * 1e-9
        self.overhead = overhead
        self.live = {}
        self.log = []
        self.next = 0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)

    def bytes_for(self, req):
        return req.particles * 32 + 1000

    def admit(self, req):
        self.next += 1
        self.live[self.next] = req
        self.log.append(("admit", req.rid, self.t))
        return self.next

    def advance(self, runs, nsteps):
        ps = sum(self.live[r].particles * n for r, n in zip(runs, nsteps))
        self.log.append(("advance", tuple(self.live[r].rid for r in runs), self.t))
        self.t += self.overhead + ps * self.rate

    def wait(self):
        pass

    def release(self, run):
        req = self.live.pop(run)
        self.log.append(("release", req.rid, self.t))
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
    assert st["n_requests"] == 60
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


def test_fifo_admission_under_tight_budget():
    reqs = _reqs(25)
    ex = FakeExecutor()
    budget = max(ex.bytes_for(r) for r in reqs)  # one large run at a time at most
    done, st = serve.schedule(reqs, ex, budget, chunk_steps=100)
    admits = [rid for ev, rid, _ in ex.log if ev == "admit"]
    assert admits == sorted(admits)


def test_request_over_budget_is_rejected():
    reqs = _reqs(3)
    ex = FakeExecutor()
    with pytest.raises(ValueError):
        serve.schedule(reqs, ex, budget_bytes=10, chunk_steps=10)


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
