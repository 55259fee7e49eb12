"""rasp_run_noalloc (queue, batch tables and survivor list in the library's
fixed device array) gives the same machines as rasp_run, on two calls in a
row, the second on a smaller batch, through the C ABI."""
import numpy as np
import pytest

from paper_2604_12902_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("status", "steps", "i", "a", "u0", "y0", "y", "mem")


def _run(R, ctx, batch, noalloc, first_pass, lds_words):
    ctx.set(R.RASP_OPT_SCHEDULE, R.RASP_SCHED_PERSISTENT)
    ctx.set(R.RASP_OPT_FIRST_PASS, first_pass)
    ctx.set(R.RASP_OPT_LDS_WORDS, lds_words)
    h = ctx.load(batch)
    if noalloc:
        R.rasp_run_noalloc(ctx.handle, h, batch.budget)
    else:
        R.rasp_run(ctx.handle, h, batch.budget)
    out = ctx.fetch(h, mem=True)
    ctx.free(h)
    return out


@pytest.mark.parametrize("first_pass,lds_words", [(0, -1), (16, 40)])
def test_noalloc_equals_run_twice_then_smaller(first_pass, lds_words):
    from paper_2604_12902_amd import rasp as R
    big = W.config3(num_vms=6000, budget=2048)
    small = W.config3(seed=7, num_vms=1500, budget=1024)
    print("noalloc: uneven 6000 then 1500 machines, first pass %d, lds words %d" % (first_pass, lds_words),
          flush=True)
    with R.Context(256 << 20) as ctx:
        for batch in (big, small):
            want = _run(R, ctx, batch, False, first_pass, lds_words)
            got = _run(R, ctx, batch, True, first_pass, lds_words)
            for k in FIELDS:
                assert np.array_equal(got[k], want[k]), (batch.N, k)
            assert int(got["steps"].sum()) > 0


def test_noalloc_rejects_a_batch_above_its_limit():
    from paper_2604_12902_amd import rasp as R
    N = (1 << 22) + 1                   # machines that halt at once: HALT, n = 4, no tape, s = 1
    b = W.Batch(W.ISA_CLASSIC, np.zeros(2 * N, np.int32), np.arange(N + 1, dtype=np.uint64) * np.uint64(2),
                np.full(N, 4, np.uint32), np.zeros(0, np.int32), np.zeros(N + 1, np.uint64),
                np.zeros(N, np.uint32), np.ones(N, np.uint32), budget=16, name="halts")
    with R.Context(1 << 30) as ctx:
        h = ctx.load(b)
        with pytest.raises(R.RaspError, match="at most 4194304 machines"):
            R.rasp_run_noalloc(ctx.handle, h, 16)
        ctx.free(h)
