"""Continuous-batching server for RASP rollout requests.

A request is a batch of machines with its own step budget.  The server keeps
the state of every admitted request resident in the device arena and advances
all of them together, one epoch at a time:

  * arrivals are queued in arrival order;
  * at every epoch boundary the queue head is admitted while the summed arena
    footprint of admitted requests stays under the cap (and at most 64 batches
    share a launch);
  * one launch (``rasp_run_multi``) advances every admitted request by
    min(remaining budget, epoch) transitions -- runs compose, so the result is
    the same as running each request alone for its whole budget;
  * a request whose budget is spent, or whose machines have all reached a
    fixed point, is retired: its outputs are fetched to the host, its arena
    space is freed and the next arrivals can be admitted.

Latency of a request = time its outputs are on the host - its arrival time.

The executor is pluggable (``RaspExecutor`` drives the library; tests use a
CPU double) and so is the clock.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import workloads as W

MAX_BATCHES_PER_LAUNCH = 64


@dataclass
class Request:
    rid: int
    arrival: float                  # seconds after the start of the stream
    config: int                     # workload family (1 plain-small, 2 plain-scale, 3 uneven)
    size: int                       # machines
    budget: int                     # transitions per machine
    seed: int
    batch: W.Batch = None
    footprint: int = 0
    handle: int = 0
    remaining: int = 0
    admitted: float = math.nan
    done: float = math.nan
    result: dict = None
    steps: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_batch(config: int, size: int, budget: int, seed: int) -> W.Batch:
    if config == 1:
        b = W.config1(seed=seed, num_vms=size)
    elif config == 2:
        b = W.config2(seed=seed, num_vms=size)
    elif config == 3:
        b = W.config3(seed=seed, num_vms=size, budget=budget)
    else:
        raise ValueError(config)
    b.budget = budget
    return b


def poisson_requests(n: int, qps: float, seed: int = 4, size_lo: int = 1024,
                     size_hi: int = 262144, budget_lo: int = 4096, budget_hi: int = 65536,
                     configs=(1, 2, 3), generate: bool = True) -> list:
    """n requests with exponential inter-arrival times at rate qps; sizes and
    budgets log-uniform on [lo, hi]; family uniform over `configs`.  Draw
    order: inter-arrival gaps, families, sizes, budgets; request r's machines
    come from seed * 1000003 + r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    fam = np.asarray(configs)[rng.integers(0, len(configs), n)]
    sizes = W.log_uniform_int(rng, size_lo, size_hi, n)
    budgets = W.log_uniform_int(rng, budget_lo, budget_hi, n)
    reqs = []
    for r in range(n):
        q = Request(r, float(arrivals[r]), int(fam[r]), int(sizes[r]), int(budgets[r]),
                    seed * 1000003 + r)
        if generate:
            q.batch = make_batch(q.config, q.size, q.budget, q.seed)
        reqs.append(q)
    return reqs


class RaspExecutor:
    """Drives librasp through its binding (one context, one stream)."""

    def __init__(self, ctx):
        from . import rasp as R
        self.R = R
        self.ctx = ctx

    def footprint(self, batch) -> int:
        return self.R.rasp_batch_footprint(self.R.make_desc(batch))

    def load(self, batch) -> int:
        return self.ctx.load(batch)

    def run(self, handles, budgets) -> None:
        self.R.rasp_run_multi(self.ctx.handle, handles, budgets)

    def running(self, handles) -> np.ndarray:
        return self.R.rasp_running_counts(self.ctx.handle, handles)

    def fetch(self, handle) -> dict:
        return self.ctx.fetch(handle, digest=True)

    def free(self, handle) -> None:
        self.ctx.free(handle)


@dataclass
class ServeStats:
    requests: int
    wall_s: float
    steps: int
    epochs: int
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_active: int
    max_footprint: int
    latencies_ms: list = field(default_factory=list)

    @property
    def steps_per_s(self) -> float:
        return self.steps / self.wall_s if self.wall_s > 0 else 0.0


class Server:
    def __init__(self, executor, cap_bytes: int, epoch: int = 4096,
                 clock=time.perf_counter, sleep=time.sleep, max_batches: int = MAX_BATCHES_PER_LAUNCH):
        self.ex = executor
        self.cap = int(cap_bytes)
        self.epoch = int(epoch)
        self.clock = clock
        self.sleep = sleep
        self.max_batches = max_batches

    def serve(self, requests, start=None) -> ServeStats:
        """Serve `requests`; arrivals count from `start()` (a clock value) when
        given, else from the end of the footprint pass."""
        pending = sorted(requests, key=lambda q: q.arrival)
        for q in pending:
            if q.batch is None:
                q.batch = make_batch(q.config, q.size, q.budget, q.seed)
            q.footprint = self.ex.footprint(q.batch)
            if q.footprint > self.cap:
                raise ValueError("request %d needs %d bytes, above the cap" % (q.rid, q.footprint))
        queue, active = [], []
        used = 0
        epochs = 0
        max_active = max_fp = 0
        t0 = self.clock() if start is None else start()
        k = 0
        n_done = 0
        while n_done < len(pending):
            now = self.clock() - t0
            while k < len(pending) and pending[k].arrival <= now:
                queue.append(pending[k])
                k += 1
            # admission: FIFO while the footprint cap and the launch width allow
            while queue and used + queue[0].footprint <= self.cap and len(active) < self.max_batches:
                q = queue.pop(0)
                q.handle = self.ex.load(q.batch)
                q.remaining = q.budget
                q.admitted = self.clock() - t0
                used += q.footprint
                active.append(q)
            max_active = max(max_active, len(active))
            max_fp = max(max_fp, used)
            if not active:
                if k < len(pending):
                    wait = pending[k].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                continue
            budgets = [min(q.remaining, self.epoch) for q in active]
            self.ex.run([q.handle for q in active], budgets)
            epochs += 1
            running = self.ex.running([q.handle for q in active])
            still = []
            for q, b, nrun in zip(active, budgets, running):
                q.remaining -= b
                if q.remaining == 0 or int(nrun) == 0:
                    q.result = self.ex.fetch(q.handle)
                    q.steps = int(np.asarray(q.result["steps"]).sum())
                    self.ex.free(q.handle)
                    q.done = self.clock() - t0
                    used -= q.footprint
                    n_done += 1
                else:
                    still.append(q)
            active = still
        wall = self.clock() - t0
        if not pending:
            return ServeStats(0, wall, 0, epochs, 0.0, 0.0, 0.0, 0, 0, [])
        lat = np.array([q.latency for q in pending]) * 1e3
        return ServeStats(len(pending), wall, sum(q.steps for q in pending), epochs,
                          float(np.percentile(lat, 50)), float(np.percentile(lat, 99)),
                          float(lat.mean()), max_active, max_fp, lat.tolist())


def serve_partitioned(executors, requests, cap_bytes: int, epoch: int = 4096,
                      clock=time.perf_counter) -> ServeStats:
    """Serve with one server per executor, each on its own host thread.

    On the device each executor is a context whose stream runs on its own
    share of the compute units, so the heavy tail of one partition's requests
    does not hold up another's.  Requests are dealt round-robin in arrival
    order; each partition gets an equal share of the footprint cap; all
    partitions count arrivals from one common start.  The merged statistics
    cover every request: wall time to the last one finished, steps and
    epochs summed, latency percentiles over all requests.
    """
    import threading
    k = len(executors)
    reqs = sorted(requests, key=lambda q: q.arrival)
    parts = [reqs[i::k] for i in range(k)]
    share = int(cap_bytes) // k
    barrier = threading.Barrier(k)
    lock = threading.Lock()
    shared = {}
    stats, errors = [None] * k, []

    def start():
        barrier.wait()
        with lock:
            if "t0" not in shared:
                shared["t0"] = clock()
        return shared["t0"]

    def run(i):
        try:
            stats[i] = Server(executors[i], share, epoch=epoch, clock=clock).serve(parts[i], start=start)
        except Exception as e:                          # re-raised below
            errors.append(e)
            barrier.abort()

    threads = [threading.Thread(target=run, args=(i,)) for i in range(k)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        raise errors[0]
    lat = np.array([q.latency for q in reqs]) * 1e3
    return ServeStats(len(reqs), max(st.wall_s for st in stats), sum(st.steps for st in stats),
                      sum(st.epochs for st in stats), float(np.percentile(lat, 50)),
                      float(np.percentile(lat, 99)), float(lat.mean()),
                      sum(st.max_active for st in stats), sum(st.max_footprint for st in stats),
                      lat.tolist())
