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

With an executor that has the asynchronous calls (``running_async``,
``fetch_async``) the host work overlaps the device: an epoch's running
counts are queued right behind its launch, and while it runs the server
collects the outputs of the previous epoch's retirees (fetched on the
context's copy stream) and loads new arrivals; it waits only for the counts.

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

    # asynchronous counterparts (the server overlaps host work with epochs)
    def running_async(self, handles):
        return self.R.rasp_running_counts_async(self.ctx.handle, handles)

    def running_wait(self, ticket) -> np.ndarray:
        return self.R.rasp_running_counts_wait(self.ctx.handle, ticket)

    def fetch_async(self, handle):
        info = self.R.rasp_batch_info(self.ctx.handle, handle)
        dst = self.R.pinned_outputs(info)
        self.R.rasp_fetch_outputs_async(self.ctx.handle, handle, dst)
        return (handle, info, dst)

    def fetch_wait(self, token) -> dict:
        handle, info, dst = token
        self.R.rasp_sync(self.ctx.handle, handle)
        return self.R.outputs_as_numpy(dst, info)


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
        queue, active, fetching = [], [], []
        used = 0
        epochs = 0
        max_active = max_fp = 0
        t0 = self.clock() if start is None else start()
        k = 0
        n_done = 0
        asyn = hasattr(self.ex, "running_async")

        def arrive():
            nonlocal k
            now = self.clock() - t0
            while k < len(pending) and pending[k].arrival <= now:
                queue.append(pending[k])
                k += 1

        def admit():
            # FIFO while the footprint cap and the launch width allow
            nonlocal used, max_active, max_fp
            while queue and used + queue[0].footprint <= self.cap and len(active) < self.max_batches:
                q = queue.pop(0)
                q.handle = self.ex.load(q.batch)
                q.remaining = q.budget
                q.admitted = self.clock() - t0
                used += q.footprint
                active.append(q)
            max_active = max(max_active, len(active))
            max_fp = max(max_fp, used)

        def finish(q, result):
            # outputs on the host: the request is done, its space free
            nonlocal used, n_done
            q.result = result
            q.steps = int(np.asarray(q.result["steps"]).sum())
            self.ex.free(q.handle)
            q.done = self.clock() - t0
            used -= q.footprint
            n_done += 1

        def collect():
            for q, token in fetching:
                finish(q, self.ex.fetch_wait(token))
            fetching.clear()

        while n_done < len(pending):
            arrive()
            admit()
            if not active:
                if fetching:
                    collect()
                    continue
                if k < len(pending):
                    wait = pending[k].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                continue
            launched = list(active)
            budgets = [min(q.remaining, self.epoch) for q in launched]
            self.ex.run([q.handle for q in launched], budgets)
            epochs += 1
            if asyn:
                ticket = self.ex.running_async([q.handle for q in launched])
                # while the epoch runs: the previous retirees' outputs, then
                # the arrivals their space admits (loaded behind the epoch)
                collect()
                arrive()
                admit()
                running = self.ex.running_wait(ticket)
            else:
                running = self.ex.running([q.handle for q in launched])
            retired = set()
            for q, b, nrun in zip(launched, budgets, running):
                q.remaining -= b
                if q.remaining == 0 or int(nrun) == 0:
                    retired.add(id(q))
                    if asyn:
                        fetching.append((q, self.ex.fetch_async(q.handle)))
                    else:
                        finish(q, self.ex.fetch(q.handle))
            active[:] = [q for q in active if id(q) not in retired]
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
