"""Serving on the GPU: requests that arrive while others run are admitted as
arena space frees up, share launches, and each result is bit-identical to the
same request run alone (and to the oracle)."""
import numpy as np
import pytest

import oracle
from paper_2604_12902_amd import serving

pytestmark = pytest.mark.gpu


def test_served_results_equal_standalone_runs():
    import torch
    from paper_2604_12902_amd import rasp as R
    assert torch.cuda.is_available()
    reqs = serving.poisson_requests(14, qps=400.0, seed=11, size_lo=1024, size_hi=20000,
                                    budget_lo=256, budget_hi=4096)
    # and one request at the largest size and budget of the serving stream:
    # 262,144 uneven machines, budget 65,536, arriving among the others
    big = serving.Request(14, reqs[5].arrival, 3, 262144, 65536, 11 * 1000003 + 14)
    big.batch = serving.make_batch(big.config, big.size, big.budget, big.seed)
    reqs.append(big)
    ctx = R.Context(6 << 30)
    ex = serving.RaspExecutor(ctx)
    fps = sorted(ex.footprint(q.batch) for q in reqs)
    cap = sum(fps[-3:])                                  # at most ~3 large requests resident
    print("case: serving 15 requests (one of 262144 machines, budget 65536) cap=%d" % cap, flush=True)
    stats = serving.Server(ex, cap, epoch=512).serve(reqs)
    assert stats.requests == 15 and stats.max_footprint <= cap and stats.max_active >= 2
    alone = R.Context(6 << 30)
    for q in reqs:
        h = alone.load(q.batch)
        alone.run(h, q.budget)
        got = alone.fetch(h, digest=True)
        alone.free(h)
        for k in ("status", "steps", "i", "a", "u0", "y0", "y", "mem_digest"):
            assert np.array_equal(np.asarray(q.result[k]), got[k]), (q.rid, k)
    # and a sample of machines of the three largest requests against the oracle
    for q in sorted(reqs, key=lambda q: -q.size)[:3]:
        idx = np.arange(0, q.batch.N, 97)
        want = oracle.run(q.batch.subset(idx), q.budget, threads=8)
        for k in ("status", "steps", "i", "a", "u0", "y0"):
            assert np.array_equal(np.asarray(q.result[k])[idx], getattr(want, k)), (q.rid, k)
    alone.close()
    ctx.close()


def test_beaver_search_on_the_served_path_matches_the_oracle():
    """App. B's search on the GPU (L = 120, all arrays zero, w = 29): the
    reported busiest beavers, halting count and tau_h decades equal what the
    oracle gives on the same sampled programs."""
    import torch
    from paper_2604_12902_amd import rasp as R, search, workloads as W
    assert torch.cuda.is_available()
    seed, rounds, batch, L, w, tau_max, keep = 7, 2, 3000, 120, 29, 20000, 8
    print("case: beaver search rounds=%d batch=%d L=%d w=%d tau_max=%d" % (rounds, batch, L, w, tau_max),
          flush=True)
    ctx = R.Context(1 << 30)
    res = search.search(serving.RaspExecutor(ctx), rounds=rounds, batch=batch, L=L, w=w,
                        tau_max=tau_max, keep=keep, seed=seed, cap_bytes=(1 << 30) - (64 << 20))
    ctx.close()
    halting, dec, run = [], {}, 0
    for r in range(rounds):
        progs, idx = [], []
        for v in range(batch):
            words = search.lower(search.program_source(seed, r, batch, v, L))
            if words is not None:
                progs.append(words)
                idx.append(v)
        b = W.from_programs(W.ISA_WORD, progs, search.BB_N, None, ell=search.BB_ELL, s=search.BB_S)
        st = oracle.run(b, tau_max, w=w, threads=8)
        run += len(idx)
        for k, v in enumerate(idx):
            if st.status[k] == oracle.HALTED:
                t = int(st.steps[k])
                halting.append((t, r, v))
                d = int(np.floor(np.log10(t))) if t > 0 else -1
                dec[d] = dec.get(d, 0) + 1
    assert res.programs == run and res.halted == len(halting)
    assert [(t, r, v) for t, r, v, _ in res.best] == sorted(halting, key=lambda e: (-e[0], e[1], e[2]))[:keep]
    assert res.decades == dec


def test_async_running_counts_and_fetch_equal_the_waiting_calls():
    """rasp_running_counts_async / _wait give what rasp_running_counts gives;
    at most four tickets are in flight (a fifth request drops the oldest);
    an asynchronous fetch into pinned buffers equals the waiting fetch, a
    later run of the batch is ordered after it, and the batch can be freed
    with the fetch still in flight."""
    import torch
    from paper_2604_12902_amd import rasp as R, workloads as W
    assert torch.cuda.is_available()
    print("case: async counts and fetch", flush=True)
    bs = [W.config3(seed=40 + t, num_vms=3000 + 1000 * t, budget=4096) for t in range(3)]
    ctx = R.Context(1 << 30)
    hs = [ctx.load(b) for b in bs]
    ctx.run_multi(hs, [300, 300, 300])
    want = R.rasp_running_counts(ctx.handle, hs)
    tickets = [R.rasp_running_counts_async(ctx.handle, hs) for _ in range(5)]
    with pytest.raises(R.RaspError):
        R.rasp_running_counts_wait(ctx.handle, tickets[0])          # dropped by the fifth
    for t in tickets[1:]:
        assert np.array_equal(R.rasp_running_counts_wait(ctx.handle, t), want)
    with pytest.raises(R.RaspError):
        R.rasp_running_counts_wait(ctx.handle, tickets[1])          # claimed once
    for h in hs:
        info = R.rasp_batch_info(ctx.handle, h)
        dst = R.pinned_outputs(info)
        R.rasp_fetch_outputs_async(ctx.handle, h, dst)
        ctx.sync(h)
        got = R.outputs_as_numpy(dst, info)
        ref = ctx.fetch(h, digest=True)
        for k in ("status", "steps", "i", "a", "u0", "y0", "y", "mem_digest"):
            assert np.array_equal(got[k], ref[k]), (h, k)
    # an asynchronous fetch, then a run: the fetch sees the state before it
    h = hs[0]
    info = R.rasp_batch_info(ctx.handle, h)
    before = ctx.fetch(h, digest=True)
    dst = R.pinned_outputs(info)
    R.rasp_fetch_outputs_async(ctx.handle, h, dst)
    ctx.run(h, 2000)
    ctx.sync(h)
    got = R.outputs_as_numpy(dst, info)
    for k in ("steps", "i", "a", "mem_digest"):
        assert np.array_equal(got[k], before[k]), k
    after = ctx.fetch(h, digest=True)
    assert after["steps"].sum() > before["steps"].sum()
    # free with a fetch in flight
    dst2 = R.pinned_outputs(R.rasp_batch_info(ctx.handle, hs[1]))
    R.rasp_fetch_outputs_async(ctx.handle, hs[1], dst2)
    ctx.free(hs[1])
    ctx.free(hs[0])
    ctx.free(hs[2])
    ctx.close()
