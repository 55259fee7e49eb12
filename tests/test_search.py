"""The busy-beaver search driver (App. B) and its Fig. 1b statistics, on the
CPU: the serving loop runs over a test double whose machines are advanced by
the oracle at the batch's word width, and every reported figure is compared
with the oracle run directly on the same programs."""
import numpy as np

import oracle
from paper_2604_12902_amd import search, workloads as W


class OracleExecutor:
    def __init__(self):
        self.states, self.next = {}, 1

    def footprint(self, batch):
        return 64 * batch.N + 4 * batch.footprint_words()

    def load(self, batch):
        h = self.next
        self.next += 1
        self.states[h] = oracle.init(batch, w=batch.word_bits)
        return h

    def run(self, handles, budgets):
        for h, b in zip(handles, budgets):
            oracle.advance(self.states[h], b)

    def running(self, handles):
        return np.array([int((self.states[h].status == 0).sum()) for h in handles])

    def fetch(self, h):
        st = self.states[h]
        return dict(status=st.status.copy(), steps=st.steps.copy())

    def free(self, h):
        del self.states[h]


def _direct(seed, rounds, batch, L, w, tau_max):
    """(tau_h, round, index) of every halting program, programs run, skipped."""
    out, run, skipped = [], 0, 0
    for r in range(rounds):
        progs, idx = [], []
        for v in range(batch):
            words = search.lower(search.program_source(seed, r, batch, v, L))
            if words is None:
                skipped += 1
                continue
            progs.append(words)
            idx.append(v)
        b = W.from_programs(W.ISA_WORD, progs, search.BB_N, None, ell=search.BB_ELL, s=search.BB_S)
        st = oracle.run(b, tau_max, w=w)
        run += len(idx)
        for k, v in enumerate(idx):
            if st.status[k] == oracle.HALTED:
                out.append((int(st.steps[k]), r, v))
    return out, run, skipped


def test_search_reports_what_the_oracle_gives():
    # L = 200: a few programs do not fit n = 250 and are skipped
    seed, rounds, batch, L, w, tau_max, keep = 3, 2, 250, 200, 29, 4000, 6
    res = search.search(OracleExecutor(), rounds=rounds, batch=batch, L=L, w=w, tau_max=tau_max,
                        keep=keep, seed=seed)
    halting, run, skipped = _direct(seed, rounds, batch, L, w, tau_max)
    assert res.programs == run and res.skipped == skipped > 0 and run + skipped == rounds * batch
    assert res.halted == len(halting) and 0 < res.halted < run
    want = sorted(halting, key=lambda e: (-e[0], e[1], e[2]))[:keep]
    assert [(t, r, v) for t, r, v, _ in res.best] == want
    for t, r, v, src in res.best:
        assert src == search.program_source(seed, r, batch, v, L)
    dec = {}
    for t, _, _ in halting:
        d = int(np.floor(np.log10(t))) if t > 0 else -1
        dec[d] = dec.get(d, 0) + 1
    assert res.decades == dec


def test_search_is_seeded_and_rounds_differ():
    a = search.program_source(0, 0, 100, 7, 120)
    assert a == search.program_source(0, 0, 100, 7, 120)
    assert a != search.program_source(0, 1, 100, 7, 120)
    assert a != search.program_source(1, 0, 100, 7, 120)
    assert len(a.split()) == 120


def test_app_b_beavers_lower_to_the_search_machine():
    """The three App. B listings (L = 120) fit the search machine, and their
    words under ``search.lower`` are the ones the halting-number pins use."""
    import json
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(gold, "busy_beavers.json")) as f:
        spec = json.load(f)
    for p in spec["programs"]:
        with open(os.path.join(gold, p["file"])) as f:
            words = search.lower(f.read())
        assert words is not None
        b = W.from_programs(W.ISA_WORD, [words], search.BB_N, None, ell=search.BB_ELL, s=search.BB_S)
        st = oracle.run(b, 10 ** 6, w=29)
        assert int(st.status[0]) == oracle.HALTED and int(st.steps[0]) == p["tau_h"]
