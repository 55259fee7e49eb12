"""Busy-beaver search (App. B) and the halting-probability estimate of Sec. 3
(Fig. 1b), run on the device through the serving loop.

Each round samples `batch` programs uniformly from the Sec. 2.2 snippets of
exactly L terminals (``grammar.sample_program``; program v of round r is drawn
from Python's Mersenne Twister seeded with seed * 2^40 + r * batch + v),
lowers them by the Sec. 2.2 rules with every array starting at zero -- no
read prologue, so ipt, scr and opt are all 0s, App. B's search setting -- and
submits the round as one request to ``serving.Server`` with budget tau_max
at word width w.  Programs whose code and data do not fit n words are
counted and skipped.

From the fetched halting numbers it keeps the `keep` halting programs with
the largest tau_h (App. B's "busiest beavers"), and accumulates the Fig. 1b
quantities: the fraction of sampled programs that reach a fixed point before
tau_max, and the number of halting programs per decade of tau_h.

usage: python -m paper_2604_12902_amd.search [--rounds R] [--batch B] [--L L]
           [--w W] [--tau-max T] [--keep K] [--seed S] [--workers J]
"""
from __future__ import annotations

import argparse
import random
import time
from dataclasses import dataclass, field

import numpy as np

from . import dsl, grammar, serving
from . import workloads as W

# the machine of App. B's search (n, l, s and scr size as in Sec. 3)
BB_N, BB_ELL, BB_S, BB_MU = 250, 10, 2, 10


@dataclass
class SearchResult:
    programs: int = 0                 # programs run (fitting n)
    skipped: int = 0                  # sampled programs that did not fit n words
    halted: int = 0                   # reached a fixed point before tau_max
    steps: int = 0                    # transitions retired in all
    seconds: float = 0.0              # wall time of the served runs
    best: list = field(default_factory=list)        # [(tau_h, round, index, source)], largest first
    decades: dict = field(default_factory=dict)     # floor(log10 tau_h) -> halting programs

    @property
    def halting_fraction(self) -> float:
        return self.halted / self.programs if self.programs else 0.0


def program_source(seed: int, rnd: int, batch: int, index: int, L: int) -> str:
    return grammar.sample_program(L, random.Random(seed * (1 << 40) + rnd * batch + index))


def lower(src: str, n: int = BB_N, ell: int = BB_ELL, s: int = BB_S, mu: int = BB_MU):
    """Program words of `src` with all arrays zero, or None when it does not fit n."""
    pairs, lay = dsl.lower_word(dsl.parse(src), ell=ell, s=s, mu=mu)
    if 2 * len(pairs) + lay.data_words > n:
        return None
    return dsl.flatten(pairs)


def _round_chunk(job):
    seed, rnd, batch, start, stop, L = job
    out = []
    for v in range(start, stop):
        words = lower(program_source(seed, rnd, batch, v, L))
        out.append((v, words))
    return out


def round_batch(seed: int, rnd: int, batch: int, L: int, w: int, tau_max: int, pool=None):
    """(Batch of the fitting programs of round `rnd`, their indices in the round, skipped)."""
    chunk = 2048
    jobs = [(seed, rnd, batch, a, min(batch, a + chunk), L) for a in range(0, batch, chunk)]
    parts = pool.map(_round_chunk, jobs) if pool is not None else [_round_chunk(j) for j in jobs]
    idx, progs = [], []
    for part in parts:
        for v, words in part:
            if words is not None:
                idx.append(v)
                progs.append(words)
    b = W.from_programs(W.ISA_WORD, progs, BB_N, None, ell=BB_ELL, s=BB_S, budget=tau_max,
                        name="beaver search round %d" % rnd)
    b.word_bits = w
    return b, np.array(idx, dtype=np.int64), batch - len(idx)


def collect(res: SearchResult, rnd: int, idx, status, steps, sources, keep: int) -> None:
    """Fold one round's fetched status and steps into `res`."""
    status = np.asarray(status)
    steps = np.asarray(steps).astype(np.int64)
    halted = status == 1
    res.programs += len(idx)
    res.halted += int(halted.sum())
    res.steps += int(steps.sum())
    for t in steps[halted]:
        d = int(np.floor(np.log10(t))) if t > 0 else -1
        res.decades[d] = res.decades.get(d, 0) + 1
    order = np.argsort(-steps[halted], kind="stable")[:keep]
    hv = np.flatnonzero(halted)[order]
    cand = res.best + [(int(steps[k]), rnd, int(idx[k]), sources(int(idx[k]))) for k in hv]
    cand.sort(key=lambda e: (-e[0], e[1], e[2]))
    res.best = cand[:keep]


def search(executor, rounds: int = 4, batch: int = 65536, L: int = 120, w: int = 29,
           tau_max: int = 10 ** 6, keep: int = 8, seed: int = 0, cap_bytes: int = 200 << 30,
           epoch: int = 1 << 20, workers: int = 1, log=None) -> SearchResult:
    """Run `rounds` rounds of `batch` sampled programs through a serving loop
    over `executor` (``serving.RaspExecutor`` on the device)."""
    res = SearchResult()
    pool = None
    if workers > 1:
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(workers)
    try:
        for rnd in range(rounds):
            b, idx, skipped = round_batch(seed, rnd, batch, L, w, tau_max, pool)
            res.skipped += skipped
            req = serving.Request(rid=rnd, arrival=0.0, config=0, size=b.N, budget=tau_max,
                                  seed=seed, batch=b)
            srv = serving.Server(executor, cap_bytes, epoch=epoch)
            t0 = time.perf_counter()
            srv.serve([req])
            res.seconds += time.perf_counter() - t0
            collect(res, rnd, idx, req.result["status"], req.result["steps"],
                    lambda v, r=rnd: program_source(seed, r, batch, v, L), keep)
            if log:
                log("search: round %d: %d programs, %d halted, best tau_h %s" % (
                    rnd, len(idx), int((np.asarray(req.result["status"]) == 1).sum()),
                    res.best[0][0] if res.best else None))
    finally:
        if pool is not None:
            pool.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--rounds", type=int, default=4)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--L", type=int, default=120)
    ap.add_argument("--w", type=int, default=29)
    ap.add_argument("--tau-max", type=int, default=10 ** 6)
    ap.add_argument("--keep", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=1)
    ap.add_argument("--arena-gb", type=float, default=8.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default knobs instead of tuning on round 0")
    args = ap.parse_args()
    import torch
    from . import rasp as R
    assert torch.cuda.is_available(), "the search runs on the device"
    ctx = R.Context(int(args.arena_gb * (1 << 30)))
    try:
        if not args.no_autotune:
            b, _, _ = round_batch(args.seed, 0, args.batch, args.L, args.w, args.tau_max)
            h = ctx.load(b)
            print("search: autotune chose %s" % R.rasp_autotune(ctx.handle, h, args.tau_max), flush=True)
            ctx.free(h)
        res = search(serving.RaspExecutor(ctx), rounds=args.rounds, batch=args.batch, L=args.L,
                     w=args.w, tau_max=args.tau_max, keep=args.keep, seed=args.seed,
                     cap_bytes=int(args.arena_gb * (1 << 30)) - (256 << 20), workers=args.workers,
                     log=lambda s: print(s, flush=True))
    finally:
        ctx.close()
    print("search: %d programs (%d skipped: do not fit n = %d), %d halt before tau_max = %d "
          "(fraction %.4f); %.3e transitions in %.2f s (%.3e /s)" % (
              res.programs, res.skipped, BB_N, res.halted, args.tau_max, res.halting_fraction,
              res.steps, res.seconds, res.steps / max(res.seconds, 1e-9)))
    print("search: halting programs per decade of tau_h: %s" % dict(sorted(res.decades.items())))
    for t, rnd, v, src in res.best:
        print("search: tau_h = %d (round %d, program %d)\n%s" % (t, rnd, v, src))


if __name__ == "__main__":
    main()
