"""The continuous-batching scheduler, on the CPU with a test double for the
library (machines advanced by the oracle) and a simulated clock."""
import numpy as np

import oracle
from paper_2604_12902_amd import serving, workloads as W


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += d


class OracleExecutor:
    """Test double: keeps oracle states, charges simulated time per launch and
    records the footprint in use, to check the admission rule."""

    def __init__(self, clock, cap):
        self.clock, self.cap = clock, cap
        self.states, self.fp, self.next = {}, {}, 1
        self.used = self.max_used = 0
        self.launches = []

    def footprint(self, batch):
        return 64 * batch.N + 4 * batch.footprint_words()

    def load(self, batch):
        h = self.next
        self.next += 1
        self.states[h] = oracle.init(batch)
        self.fp[h] = self.footprint(batch)
        self.used += self.fp[h]
        self.max_used = max(self.max_used, self.used)
        assert self.used <= self.cap
        return h

    def run(self, handles, budgets):
        assert len(handles) <= serving.MAX_BATCHES_PER_LAUNCH
        self.launches.append(list(handles))
        for h, b in zip(handles, budgets):
            oracle.advance(self.states[h], b)
        self.clock.t += 1e-3 * len(handles)

    def running(self, handles):
        return np.array([int((self.states[h].status == 0).sum()) for h in handles])

    def fetch(self, h):
        st = self.states[h]
        return dict(status=st.status.copy(), steps=st.steps.copy(), i=st.i.copy(), a=st.a.copy(),
                    u0=st.u0.copy(), y0=st.y0.copy(), y=st.Y.copy(), mem_digest=oracle.digest(st))

    def free(self, h):
        self.used -= self.fp.pop(h)
        del self.states[h]


def small_requests(n=14, qps=300.0):
    return serving.poisson_requests(n, qps, seed=9, size_lo=16, size_hi=300, budget_lo=40,
                                    budget_hi=700, generate=True)


def test_every_request_completes_with_its_standalone_result():
    clock = FakeClock()
    reqs = small_requests()
    cap = 3 * max(64 * q.batch.N + 4 * q.batch.footprint_words() for q in reqs)
    ex = OracleExecutor(clock, cap)
    stats = serving.Server(ex, cap, epoch=100, clock=clock, sleep=clock.sleep).serve(reqs)
    assert stats.requests == len(reqs)
    assert ex.max_used <= cap and not ex.states
    for q in reqs:
        want = oracle.run(q.batch, q.budget)
        for k in ("status", "steps", "i", "a", "u0", "y0"):
            assert np.array_equal(q.result[k], getattr(want, k)), (q.rid, k)
        assert np.array_equal(q.result["y"], want.Y)
        assert np.array_equal(q.result["mem_digest"], oracle.digest(want))
        assert q.done >= q.admitted >= q.arrival
    assert stats.p99_ms >= stats.p50_ms > 0


def test_requests_overlap_and_admission_is_fifo_under_the_cap():
    clock = FakeClock()
    reqs = small_requests(n=20, qps=2000.0)
    cap = 2 * max(64 * q.batch.N + 4 * q.batch.footprint_words() for q in reqs)
    ex = OracleExecutor(clock, cap)
    serving.Server(ex, cap, epoch=50, clock=clock, sleep=clock.sleep).serve(reqs)
    # several requests shared launches (continuous batching, not a queue alone)
    assert max(len(l) for l in ex.launches) >= 2
    order = sorted(reqs, key=lambda q: q.admitted)
    assert [q.rid for q in order] == sorted(q.rid for q in reqs)     # FIFO
    # a request admitted while another was in flight shares its launches
    shared = sum(1 for l in ex.launches if len(l) > 1)
    assert shared > 0


def test_poisson_stream_is_seeded():
    a = serving.poisson_requests(30, 10.0, seed=3, generate=False)
    b = serving.poisson_requests(30, 10.0, seed=3, generate=False)
    assert [(q.arrival, q.size, q.budget, q.config) for q in a] == \
           [(q.arrival, q.size, q.budget, q.config) for q in b]
    sizes = np.array([q.size for q in a])
    assert sizes.min() >= 1024 and sizes.max() <= 262144
    gaps = np.diff([q.arrival for q in serving.poisson_requests(4000, 10.0, seed=5, generate=False)])
    assert 0.09 < gaps.mean() < 0.11


class LockedOracleExecutor:
    """Test double for one partition: oracle states, and a record of the
    footprint in use (each partition has its own)."""

    def __init__(self, cap):
        self.cap, self.states, self.fp, self.next = cap, {}, {}, 1
        self.used = self.max_used = 0

    def footprint(self, batch):
        return 64 * batch.N + 4 * batch.footprint_words()

    def load(self, batch):
        h = self.next
        self.next += 1
        self.states[h] = oracle.init(batch)
        self.fp[h] = self.footprint(batch)
        self.used += self.fp[h]
        self.max_used = max(self.max_used, self.used)
        assert self.used <= self.cap
        return h

    def run(self, handles, budgets):
        for h, b in zip(handles, budgets):
            oracle.advance(self.states[h], b)

    def running(self, handles):
        return np.array([int((self.states[h].status == 0).sum()) for h in handles])

    def fetch(self, h):
        st = self.states[h]
        return dict(status=st.status.copy(), steps=st.steps.copy(), i=st.i.copy(), a=st.a.copy(),
                    u0=st.u0.copy(), y0=st.y0.copy(), y=st.Y.copy(), mem_digest=oracle.digest(st))

    def free(self, h):
        self.used -= self.fp.pop(h)
        del self.states[h]


def test_partitioned_serving_deals_requests_and_keeps_each_share_of_the_cap():
    reqs = small_requests(n=18, qps=4000.0)
    k = 3
    share = 2 * max(64 * q.batch.N + 4 * q.batch.footprint_words() for q in reqs)
    exs = [LockedOracleExecutor(share) for _ in range(k)]
    stats = serving.serve_partitioned(exs, reqs, k * share, epoch=60)
    assert stats.requests == len(reqs) and stats.p99_ms >= stats.p50_ms > 0
    for ex in exs:
        assert 0 < ex.max_used <= share and not ex.states
    order = sorted(reqs, key=lambda q: q.arrival)
    for i, q in enumerate(order):
        want = oracle.run(q.batch, q.budget)
        for f in ("status", "steps", "i", "a", "u0", "y0"):
            assert np.array_equal(q.result[f], getattr(want, f)), (q.rid, f)
        assert np.array_equal(q.result["mem_digest"], oracle.digest(want))
        assert q.done >= q.admitted >= q.arrival
    assert stats.steps == sum(int(q.result["steps"].sum()) for q in reqs)


class AsyncOracleExecutor(OracleExecutor):
    """The double with the asynchronous calls: running counts come back
    through a ticket, outputs through a fetch token; a request whose fetch is
    in flight must not be run again, and is freed only after its fetch was
    collected."""

    def __init__(self, clock, cap):
        super().__init__(clock, cap)
        self.tickets, self.fetching, self.collected = {}, {}, set()
        self.next_ticket = 1

    def run(self, handles, budgets):
        assert not (set(handles) & set(self.fetching)), "a request with a fetch in flight was run"
        super().run(handles, budgets)

    def running_async(self, handles):
        t = self.next_ticket
        self.next_ticket += 1
        self.tickets[t] = self.running(handles)
        return t

    def running_wait(self, ticket):
        return self.tickets.pop(ticket)

    def fetch_async(self, h):
        self.fetching[h] = self.fetch(h)
        return h

    def fetch_wait(self, token):
        self.collected.add(token)
        return self.fetching.pop(token)

    def free(self, h):
        assert h in self.collected and h not in self.fetching
        super().free(h)


def test_overlapped_serving_gives_the_standalone_results():
    clock = FakeClock()
    reqs = small_requests(n=20, qps=2000.0)
    cap = 2 * max(64 * q.batch.N + 4 * q.batch.footprint_words() for q in reqs)
    ex = AsyncOracleExecutor(clock, cap)
    stats = serving.Server(ex, cap, epoch=50, clock=clock, sleep=clock.sleep).serve(reqs)
    assert stats.requests == len(reqs) and ex.max_used <= cap
    assert not ex.states and not ex.fetching and not ex.tickets
    for q in reqs:
        want = oracle.run(q.batch, q.budget)
        for k in ("status", "steps", "i", "a", "u0", "y0"):
            assert np.array_equal(q.result[k], getattr(want, k)), (q.rid, k)
        assert np.array_equal(q.result["mem_digest"], oracle.digest(want))
        assert q.done >= q.admitted >= q.arrival
    order = sorted(reqs, key=lambda q: q.admitted)
    assert [q.rid for q in order] == sorted(q.rid for q in reqs)     # FIFO
    assert max(len(l) for l in ex.launches) >= 2
