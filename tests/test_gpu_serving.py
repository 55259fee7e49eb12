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
    ctx = R.Context(1 << 30)
    ex = serving.RaspExecutor(ctx)
    fps = sorted(ex.footprint(q.batch) for q in reqs)
    cap = sum(fps[-3:])                                  # at most ~3 large requests resident
    print("case: serving 14 requests cap=%d" % cap, flush=True)
    stats = serving.Server(ex, cap, epoch=512).serve(reqs)
    assert stats.requests == 14 and stats.max_footprint <= cap and stats.max_active >= 2
    alone = R.Context(1 << 30)
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
