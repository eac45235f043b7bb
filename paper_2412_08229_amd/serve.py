"""Continuous-batching solve server for periodic-box lattice Boltzmann runs.

Requests (a flow, a grid, a Reynolds number, a step count and a precision
class) arrive over time.  The server keeps every admitted solve resident on
the device, admits new ones as soon as a slot and enough device memory are
free (FIFO, by the footprint ``nco_lattice_bytes`` reports), and advances all
active solves together: each round is one ``nco_batch_step`` call (one grouped
dispatch per kernel kind and step) over every active lattice, so solves that
arrive while others run share the device with them.  Finished solves are
read out (float64 global sums) and freed, and their latency (arrival to
result on the host) is recorded.

The compute engine is pluggable: ``GpuEngine`` drives libnco.so; tests of the
scheduling logic use a simulated engine on the CPU.
"""
import argparse
import collections
import itertools
import json
import math
import sys
import time
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import inputs
from .lattice import batch_step

GRIDS = (32, 64, 96, 128, 192)
CLASSES = {"f32": ("f32", "f32_mfma"), "bf16": ("bf16", "bf16")}   # storage, network arithmetic
U0 = 0.1 / math.sqrt(3.0)                                          # Ma = 0.1


@dataclass
class Request:
    rid: int
    arrival: float
    n: int
    re: float
    steps: int
    flow: str            # "tgv" or "turb"
    cls: str             # "f32" or "bf16"
    admitted: float = -1.0
    finished: float = -1.0
    status: str = "pending"
    result: dict = field(default_factory=dict)

    @property
    def work(self):
        return self.n ** 3 * self.steps

    @property
    def latency(self):
        return self.finished - self.arrival


def poisson_requests(count, rate, seed, grids=GRIDS, re=(400.0, 3000.0), steps=(500, 2000),
                     classes=("f32", "bf16")):
    """Seeded Poisson arrivals (rate per second) with uniformly drawn grid,
    Reynolds number, step count, flow (Taylor-Green or decaying turbulence)
    and precision class."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        out.append(Request(rid=i, arrival=t, n=int(rng.choice(grids)), re=float(rng.uniform(*re)),
                           steps=int(rng.integers(steps[0], steps[1] + 1)),
                           flow=("tgv", "turb")[int(rng.integers(0, 2))],
                           cls=classes[int(rng.integers(0, len(classes)))]))
    return out


class GpuEngine:
    """libnco.so lattices on one stream, batched with nco_batch_step."""

    def __init__(self, width=32, seed=0, stream=None, check_every=50, mass_tol=1e-3):
        """check_every, mass_tol: the library's stability check on every
        solve (a request whose state blows up ends as "unstable")."""
        from . import _lib
        self._lib = _lib
        self.params = inputs.mlp_params(width, seed)
        self.width = width
        self.stream = stream
        self.check_every, self.mass_tol = check_every, mass_tol

    def bytes(self, req):
        storage = CLASSES[req.cls][0]
        return self._lib.nco_lattice_bytes(req.n, req.n, req.n, self._lib.STORAGE[storage])

    def prepare(self, req):
        """Host-side work of admission (initial fields), done while the
        device runs the previous round."""
        _, tau = inputs.viscosity(req.n, U0, req.re)
        if req.flow == "tgv":
            rho, u = inputs.tgv3d(req.n, U0)
        else:
            rho, u = inputs.turbulence(req.n, seed=1000 + req.rid, k0=4.0, urms=U0 / 2)
        return tau, rho, u

    def create(self, req, prep=None):
        from .lattice import Lattice
        storage, mlp = CLASSES[req.cls]
        tau, rho, u = prep if prep is not None else self.prepare(req)
        lat = Lattice((req.n, req.n, req.n), storage, "nco", tau, stream=self.stream)
        lat.set_net_weights(self.params, self.width, "tanh", mlp)
        if storage == "bf16":
            # BF16 deviations rounded stochastically (keyed by the request, so
            # a request's result does not depend on what it is served with).
            lat.set_stochastic_rounding(True, req.rid)
        lat.init_equilibrium(rho, u)
        lat.set_check(self.check_every, self.mass_tol)
        return lat

    def step_batch(self, lats, steps, overlap=None):
        """Queue one round, run ``overlap`` on the host meanwhile, then wait.
        Returns the indices of lattices whose stability check failed."""
        batch_step(lats, steps)
        if overlap is not None:
            overlap()
        unstable = []
        for i, lat in enumerate(lats):
            try:
                lat.sync()
            except self._lib.NCOError as e:
                if e.status != self._lib.NCO_E_UNSTABLE:
                    raise
                unstable.append(i)
        return unstable

    def result(self, lat):
        try:
            s = lat.global_sums()
        except self._lib.NCOError as e:
            if e.status != self._lib.NCO_E_UNSTABLE:
                raise
            return {}
        return {"mass": float(s[0]), "momentum": [float(v) for v in s[1:4]],
                "kinetic_energy": float(s[4] / lat.n)}

    def destroy(self, lat):
        lat.close()


class Server:
    """FIFO admission by device-memory budget and slots, rounds of ``chunk``
    steps over every active solve."""

    def __init__(self, engine, budget_bytes, max_slots=16, chunk=50, prep_workers=0):
        """prep_workers > 0: host-side set-up of arrived requests runs on that
        many threads, concurrently with the device rounds; 0: it runs on the
        calling thread while a round is in flight."""
        self.engine = engine
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.prep_workers = int(prep_workers)

    def run(self, requests, clock=time.perf_counter, sleep=time.sleep, log=None):
        pool = ThreadPoolExecutor(self.prep_workers) if self.prep_workers > 0 else None
        try:
            return self._run(requests, clock, sleep, log, pool)
        finally:
            if pool is not None:
                pool.shutdown(wait=True)

    def _run(self, requests, clock, sleep, log, pool):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active = []           # [request, handle, remaining steps, bytes]
        used = 0
        peak_used = 0
        t0 = clock()
        done = []
        node_steps = 0
        prepared = {}         # rid -> set-up result (or its Future)

        def prepare_arrived():
            # Set up the arrived head of the queue (at most one slot's worth
            # of requests ahead) before it is admitted.
            now = clock() - t0
            for req in itertools.islice(pending, 0, self.max_slots):
                if req.arrival > now:
                    break
                if req.rid not in prepared:
                    prepared[req.rid] = pool.submit(self.engine.prepare, req) if pool else self.engine.prepare(req)

        def ready(req, wait):
            p = prepared.get(req.rid)
            if isinstance(p, Future) and not p.done() and not wait:
                return False
            return True

        def take(req):
            p = prepared.pop(req.rid, None)
            return p.result() if isinstance(p, Future) else p

        while pending or active:
            if pool is not None:
                prepare_arrived()
            now = clock() - t0
            # Admission: the head of the queue, as long as a slot and memory are free.
            while pending and pending[0].arrival <= now and len(active) < self.max_slots:
                req = pending[0]
                nb = self.engine.bytes(req)
                if nb > self.budget:
                    pending.popleft()
                    take(req)
                    req.status, req.finished = "rejected", clock() - t0
                    done.append(req)
                    continue
                if used + nb > self.budget or not ready(req, wait=not active):
                    break
                pending.popleft()
                handle = self.engine.create(req, take(req))
                req.admitted, req.status = clock() - t0, "running"
                active.append([req, handle, req.steps, nb])
                used += nb
                peak_used = max(peak_used, used)
            if not active:
                if pending:
                    sleep(max(0.0, min(pending[0].arrival - (clock() - t0), 0.05)))
                continue
            steps = [min(self.chunk, a[2]) for a in active]
            unstable = self.engine.step_batch([a[1] for a in active], steps,
                                              overlap=None if pool else prepare_arrived)
            unstable = set(unstable or ())
            node_steps += sum(a[0].n ** 3 * s for a, s in zip(active, steps))
            still = []
            for i, (a, s) in enumerate(zip(active, steps)):
                a[2] -= s
                if a[2] > 0 and i not in unstable:
                    still.append(a)
                    continue
                req = a[0]
                if i in unstable:
                    # Failed stability check: the request ends here and frees its slot.
                    req.result, req.status = {}, "unstable"
                else:
                    res = self.engine.result(a[1])
                    req.result = res
                    vals = np.hstack([np.ravel(v) for v in res.values()]) if res else np.array([np.nan])
                    req.status = "done" if np.all(np.isfinite(vals)) else "unstable"
                req.finished = clock() - t0
                self.engine.destroy(a[1])
                used -= a[3]
                done.append(req)
                if log:
                    log("request %d (%d^3, %d steps, %s/%s) %s after %.3f s"
                        % (req.rid, req.n, req.steps, req.flow, req.cls, req.status, req.latency))
            active = still
        wall = clock() - t0
        return report(done, wall, node_steps, peak_used, self.budget)


def report(done, wall, node_steps, peak_used, budget):
    out = {"requests": len(done), "wall_s": wall, "node_steps": node_steps,
           "glups": node_steps / wall / 1e9 if wall > 0 else 0.0,
           "peak_bytes": peak_used, "budget_bytes": budget,
           "status": dict(collections.Counter(r.status for r in done)), "latency_s": {}}
    for cls in sorted({r.cls for r in done}) + ["all"]:
        lat = np.array([r.latency for r in done if r.status == "done" and (cls == "all" or r.cls == cls)])
        if len(lat):
            out["latency_s"][cls] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                     "mean": float(lat.mean()), "count": int(len(lat))}
    return out


def capacity_glups(engine, chunk=50, grids=GRIDS):
    """Aggregate GLUPS of one batch holding one solve per grid and class."""
    reqs = [Request(rid=i, arrival=0.0, n=n, re=1600.0, steps=chunk, flow="tgv", cls=c)
            for i, (n, c) in enumerate((n, c) for n in grids for c in CLASSES)]
    lats = [engine.create(r) for r in reqs]
    engine.step_batch(lats, [5] * len(lats))
    t = time.perf_counter()
    engine.step_batch(lats, [chunk] * len(lats))
    dt = time.perf_counter() - t
    for l in lats:
        engine.destroy(l)
    return sum(r.n ** 3 for r in reqs) * chunk / dt / 1e9


def main(argv=None):
    ap = argparse.ArgumentParser(description="Poisson stream of periodic-box solves on one GPU")
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--loads", default="0.5,0.9", help="offered loads, fractions of the measured capacity")
    ap.add_argument("--budgets", default="free,2",
                    help="device-memory budgets in GB ('free': 90 %% of the free memory); every load runs "
                         "with the first, the last load also with the others")
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--prep-workers", type=int, default=2)
    args = ap.parse_args(argv)
    import torch
    stream = torch.cuda.Stream()
    engine = GpuEngine(stream=stream.cuda_stream)
    free = torch.cuda.mem_get_info()[0]
    budgets = [int(0.9 * free) if b == "free" else int(float(b) * 2 ** 30) for b in args.budgets.split(",")]
    cap = capacity_glups(engine, chunk=args.chunk)
    mean_work = np.mean([n ** 3 for n in GRIDS]) * 1250.0
    print(json.dumps({"capacity_glups": cap, "mean_request_node_steps": mean_work}), flush=True)
    loads = [float(x) for x in args.loads.split(",")]
    runs = [(x, budgets[0]) for x in loads] + [(loads[-1], b) for b in budgets[1:]]
    for load, bud in runs:
        rate = load * cap * 1e9 / mean_work
        reqs = poisson_requests(args.requests, rate, args.seed)
        srv = Server(engine, bud, max_slots=args.slots, chunk=args.chunk, prep_workers=args.prep_workers)
        rep = srv.run(reqs, log=lambda s: print("# " + s, file=sys.stderr, flush=True))
        rep.update({"offered_load": load, "arrival_rate_per_s": rate})
        print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
