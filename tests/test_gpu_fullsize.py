"""Parity at the full population sizes, in the launch configuration the
benchmark times (default knobs of the persistent schedule).  Every machine's
scalars are compared where the oracle can afford the whole population;
otherwise a seeded sample of machines, which the oracle recomputes one by one
from their own programs, plus properties that hold at any size."""
import numpy as np
import pytest

import oracle
from paper_2604_12902_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_2604_12902_amd import rasp
    assert torch.cuda.is_available()
    return rasp


def _run(R, b, arena_extra=1.2, knobs=None):
    d = R.make_desc(b)
    ctx = R.Context(int(R.rasp_batch_footprint(d) * arena_extra) + (64 << 20))
    for opt, val in (knobs or {}).items():
        ctx.set(opt, val)
    h = R.rasp_load_batch(ctx.handle, d)
    ctx.run(h, b.budget)
    got = ctx.fetch(h, digest=True)
    info = ctx.info(h, steps_sum=True)
    ctx.free(h)
    ctx.close()
    return got, info


def _check_sample(b, got, idx):
    sub = b.subset(idx)
    want = oracle.run(sub, b.budget, threads=16)
    for k in ("status", "steps", "i", "a", "u0", "y0"):
        assert np.array_equal(got[k][idx], getattr(want, k)), k
    assert np.array_equal(got["mem_digest"][idx], oracle.digest(want))
    yo = np.zeros(b.N + 1, np.int64)
    np.cumsum(b.out_cap.astype(np.int64), out=yo[1:])
    for j, v in enumerate(idx):
        assert np.array_equal(got["y"][yo[v]:yo[v + 1]], want.out_of(j)), v


def test_plain_scale_every_machine(R):
    b = W.config2()
    print("case: plain-scale N=%d" % b.N, flush=True)
    got, info = _run(R, b)
    want = oracle.run(b, b.budget, threads=16)
    for k in ("status", "steps", "i", "a", "u0", "y0"):
        assert np.array_equal(got[k], getattr(want, k)), k
    assert np.array_equal(got["y"], want.Y)
    assert np.array_equal(got["mem_digest"], oracle.digest(want))
    assert info["steps_sum"] == int(want.steps.sum())


@pytest.mark.parametrize("slots", ["default", "split32"])
def test_uneven_batch_full_size_sampled(R, slots):
    """4,194,304 machines, n 64-1,024: default knobs (memories in HBM), and
    the 32-word split slots the autotuner picks for this workload."""
    b = W.config3()
    print("case: uneven N=%d slots=%s" % (b.N, slots), flush=True)
    knobs = {R.RASP_OPT_LDS_WORDS: 32} if slots == "split32" else None
    got, info = _run(R, b, knobs=knobs)
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.sort(rng.choice(b.N, 3000, replace=False))
    # include the slowest machines the GPU reports, to cover the long tail
    idx = np.unique(np.concatenate([idx, np.argsort(got["steps"])[-200:]]))
    _check_sample(b, got, idx)
    assert (got["steps"] <= b.budget).all() and (got["u0"] <= 32).all()
    assert (got["y0"] <= 16).all()
    assert info["steps_sum"] == int(got["steps"].sum())


def test_rollouts_full_size_sampled(R):
    b = W.config4()
    print("case: rollouts N=%d" % b.N, flush=True)
    got, info = _run(R, b)
    rng = np.random.Generator(np.random.PCG64(8))
    idx = np.sort(rng.choice(b.N, 400, replace=False))
    _check_sample(b, got, idx)
    # every rollout program halts well inside its budget
    assert (got["status"] == 1).all()


@pytest.mark.parametrize("slots", ["whole", "split152"])
def test_fig1_workload_sampled(R, slots):
    """The Sec. 3 evaluation's shape: uniform L = 100 programs, word RASP,
    n = 250 (not a power of two), budget 10^6; 65,536 machines, a seeded
    sample plus the first 2,000 machines.  'whole': default slots (every
    memory in LDS, 2 waves per CU); 'split152': the slots the autotuner picks
    for this workload (words 0-151 in LDS, the rest in HBM, 4 waves per CU)."""
    b = W.fig1(num_vms=1 << 16)
    print("case: fig1 N=%d slots=%s" % (b.N, slots), flush=True)
    knobs = {R.RASP_OPT_LDS_WORDS: 152} if slots == "split152" else None
    got, info = _run(R, b, knobs=knobs)
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.unique(np.concatenate([np.sort(rng.choice(b.N, 1500, replace=False)),
                                    np.arange(2000)]))
    _check_sample(b, got, idx)
    assert (got["steps"] <= b.budget).all() and (got["u0"] <= 10).all()
    assert ((got["status"] == 1) | (got["steps"] == b.budget)).all()
    assert info["steps_sum"] == int(got["steps"].sum())
