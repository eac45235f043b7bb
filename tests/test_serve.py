"""Scheduling logic of the solve server on the CPU, with a simulated engine
and a simulated clock (no device, no library)."""
import numpy as np
import pytest

from paper_2412_08229_amd import serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimEngine:
    """Advances the clock by node-steps / rate per batch; tracks live bytes."""

    def __init__(self, clock, rate=1e9, overhead=1e-4):
        self.clock, self.rate, self.overhead = clock, rate, overhead
        self.live = {}
        self.batches = []
        self.next = 0
        self.prepared = []

    def bytes(self, req):
        per = {"f32": 2 * 27 * 4, "bf16": 2 * 27 * 2}[req.cls]
        return req.n ** 3 * per + 4096

    def prepare(self, req):
        self.prepared.append(req.rid)
        return ("fields", req.rid)

    def create(self, req, prep=None):
        assert prep is None or prep == ("fields", req.rid)
        h = self.next
        self.next += 1
        self.live[h] = (req, self.bytes(req))
        return h

    def step_batch(self, handles, steps, overlap=None):
        self.batches.append(list(zip(handles, steps)))
        if overlap is not None:
            overlap()
        work = sum(self.live[h][0].n ** 3 * s for h, s in zip(handles, steps))
        self.clock.t += self.overhead + work / self.rate

    def result(self, h):
        return {"mass": float(self.live[h][0].n ** 3)}

    def destroy(self, h):
        del self.live[h]


def _run(reqs, budget, slots=16, chunk=50, rate=1e9, workers=0):
    clk = Clock()
    eng = SimEngine(clk, rate)
    peak = {"bytes": 0, "slots": 0}
    orig = eng.step_batch

    def watch(handles, steps, overlap=None):
        peak["bytes"] = max(peak["bytes"], sum(b for _, b in eng.live.values()))
        peak["slots"] = max(peak["slots"], len(handles))
        orig(handles, steps, overlap)
    eng.step_batch = watch
    rep = serve.Server(eng, budget, max_slots=slots, chunk=chunk, prep_workers=workers).run(
        reqs, clock=clk, sleep=clk.sleep)
    return rep, eng, peak


def test_poisson_requests_are_seeded_and_in_range():
    a = serve.poisson_requests(200, rate=3.0, seed=7)
    b = serve.poisson_requests(200, rate=3.0, seed=7)
    assert [(r.arrival, r.n, r.steps, r.flow, r.cls) for r in a] == [(r.arrival, r.n, r.steps, r.flow, r.cls) for r in b]
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    # Mean inter-arrival time of an exponential with rate 3: 1/3 (loose bound, 200 draws).
    assert abs(np.diff(arr).mean() - 1.0 / 3.0) < 0.08
    assert {r.n for r in a} <= set(serve.GRIDS) and {r.cls for r in a} == {"f32", "bf16"}
    assert all(500 <= r.steps <= 2000 and 400 <= r.re <= 3000 for r in a)


def test_every_request_finishes_with_its_steps():
    reqs = serve.poisson_requests(30, rate=20.0, seed=1, grids=(16, 32, 48), steps=(10, 200))
    rep, eng, _ = _run(reqs, budget=1 << 30, chunk=25)
    assert rep["status"] == {"done": 30}
    done_steps = {}
    for batch in eng.batches:
        for h, s in batch:
            done_steps[h] = done_steps.get(h, 0) + s
    assert sorted(done_steps.values()) == sorted(r.steps for r in reqs)
    assert not eng.live
    assert all(r.finished >= r.admitted >= r.arrival for r in reqs)
    assert rep["node_steps"] == sum(r.work for r in reqs)


def test_budget_and_slots_are_respected():
    reqs = [serve.Request(rid=i, arrival=0.0, n=32, re=1000.0, steps=100, flow="tgv", cls="f32") for i in range(10)]
    one = SimEngine(Clock()).bytes(reqs[0])
    rep, eng, peak = _run(reqs, budget=3 * one + 10, slots=16)
    assert peak["bytes"] <= 3 * one + 10 and peak["slots"] == 3
    assert rep["peak_bytes"] == 3 * one
    # The seven queued requests had their host-side set-up done during
    # rounds, once each.
    assert sorted(eng.prepared) == list(range(3, 10))
    rep, _, peak = _run(reqs, budget=1 << 40, slots=4)
    assert peak["slots"] == 4


def test_fifo_admission_and_rejection():
    big = serve.Request(rid=0, arrival=0.0, n=192, re=1000.0, steps=10, flow="tgv", cls="f32")
    small = [serve.Request(rid=i, arrival=0.001 * i, n=16, re=1000.0, steps=10, flow="tgv", cls="f32")
             for i in range(1, 5)]
    budget = SimEngine(Clock()).bytes(small[0]) * 2
    rep, _, _ = _run([big] + small, budget=budget)
    assert big.status == "rejected"
    assert rep["status"] == {"rejected": 1, "done": 4}
    # FIFO: requests of equal work are admitted in arrival order.
    adm = [r.admitted for r in small]
    assert adm == sorted(adm)


def test_head_of_line_waits_for_memory():
    # A large request at the head of the queue is not overtaken by later small ones.
    a = serve.Request(rid=0, arrival=0.0, n=64, re=1000.0, steps=200, flow="tgv", cls="f32")
    b = serve.Request(rid=1, arrival=0.01, n=64, re=1000.0, steps=50, flow="tgv", cls="f32")
    c = serve.Request(rid=2, arrival=0.02, n=16, re=1000.0, steps=50, flow="tgv", cls="f32")
    eng = SimEngine(Clock())
    budget = eng.bytes(a) + eng.bytes(c) + 10
    _run([a, b, c], budget=budget)
    assert b.admitted >= a.finished - 1e-12
    assert c.admitted >= b.admitted


def test_latency_percentiles_by_class():
    reqs = serve.poisson_requests(40, rate=50.0, seed=3, grids=(16, 32), steps=(10, 100))
    rep, _, _ = _run(reqs, budget=1 << 30, chunk=10, rate=1e8)
    for cls in ("f32", "bf16", "all"):
        lat = np.array([r.latency for r in reqs if cls == "all" or r.cls == cls])
        got = rep["latency_s"][cls]
        assert got["count"] == len(lat)
        assert got["p50"] == pytest.approx(np.percentile(lat, 50))
        assert got["p99"] == pytest.approx(np.percentile(lat, 99))
        assert got["p99"] >= got["p50"] > 0
    assert rep["glups"] == pytest.approx(rep["node_steps"] / rep["wall_s"] / 1e9)


def test_batching_beats_serial_latency():
    # Many small solves arriving together: one shared batch per round
    # finishes them sooner on average than one solve at a time.
    reqs = lambda: [serve.Request(rid=i, arrival=0.0, n=16, re=1000.0, steps=100, flow="tgv", cls="f32")
                    for i in range(8)]
    rep_b, _, _ = _run(reqs(), budget=1 << 30, slots=8, chunk=20)
    rep_s, _, _ = _run(reqs(), budget=1 << 30, slots=1, chunk=20)
    assert rep_b["latency_s"]["all"]["mean"] < rep_s["latency_s"]["all"]["mean"]


def test_threaded_preparation():
    reqs = serve.poisson_requests(25, rate=40.0, seed=4, grids=(16, 32), steps=(10, 80))
    clk = Clock()
    eng = SimEngine(clk)
    rep = serve.Server(eng, 1 << 30, max_slots=4, chunk=10, prep_workers=2).run(reqs, clock=clk, sleep=clk.sleep)
    assert rep["status"] == {"done": 25}
    assert sorted(eng.prepared) == list(range(25))
    adm = [r.admitted for r in sorted(reqs, key=lambda r: r.arrival)]
    assert adm == sorted(adm) and not eng.live


class UnstableEngine(SimEngine):
    """Reports request 1 unstable after its first round."""

    def step_batch(self, handles, steps, overlap=None):
        super().step_batch(handles, steps, overlap)
        return [i for i, h in enumerate(handles) if self.live[h][0].rid == 1]


def test_unstable_request_frees_its_slot():
    reqs = [serve.Request(rid=i, arrival=0.0, n=16, re=1000.0, steps=100, flow="tgv", cls="f32") for i in range(3)]
    clk = Clock()
    eng = UnstableEngine(clk)
    one = eng.bytes(reqs[0])
    rep = serve.Server(eng, 2 * one, max_slots=2, chunk=10).run(reqs, clock=clk, sleep=clk.sleep)
    assert rep["status"] == {"done": 2, "unstable": 1}
    assert reqs[1].status == "unstable" and reqs[1].result == {}
    # Its slot went to request 2 after one round, not after 100 steps.
    assert reqs[2].admitted < reqs[0].finished
    assert rep["latency_s"]["all"]["count"] == 2 and not eng.live
