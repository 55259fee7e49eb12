"""GPU parity: the HIP library against the CPU oracle, bit-exact.

Every test calls the library through its C ABI (the ctypes binding) and
compares every output field with the oracle run on the same seeded inputs.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2604_12902_amd import dsl, workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SCHEDULES = {
    "plain": dict(schedule=1),
    "persistent-hbm": dict(schedule=2, first_pass=0, lds_words=0, epoch=16),
    "persistent-lds32": dict(schedule=2, first_pass=0, lds_words=32, epoch=8),
    "firstpass-lds64": dict(schedule=2, first_pass=4, lds_words=64, epoch=32),
    "firstpass-lds16-tiny-epoch": dict(schedule=2, first_pass=1, lds_words=16, epoch=1),
}


@pytest.fixture(scope="module")
def rasp():
    import torch
    from paper_2604_12902_amd import rasp as R
    assert torch.cuda.is_available()
    return R


@pytest.fixture(scope="module")
def ctx(rasp):
    c = rasp.Context(1 << 30)
    yield c
    c.close()


def configure(ctx, rasp, sched):
    o = SCHEDULES[sched]
    ctx.set(rasp.RASP_OPT_SCHEDULE, o["schedule"])
    if "first_pass" in o:
        ctx.set(rasp.RASP_OPT_FIRST_PASS, o["first_pass"])
        ctx.set(rasp.RASP_OPT_LDS_WORDS, o["lds_words"])
        ctx.set(rasp.RASP_OPT_EPOCH, o["epoch"])


def compare(got, want: oracle.State, mem=True, idx=None):
    sl = slice(None) if idx is None else idx
    for k in ("status", "steps", "i", "a", "u0", "y0"):
        g, w = got[k], getattr(want, k)
        if idx is not None:
            g = g[idx]
        bad = np.flatnonzero(g != w)
        assert bad.size == 0, "%s differs at machines %s: gpu %s oracle %s" % (
            k, bad[:5], g[bad[:5]], w[bad[:5]])
    if idx is None:
        assert np.array_equal(got["y"], want.Y), "output words differ"
        if mem:
            assert np.array_equal(got["mem"], want.mem), "memory differs"
    del sl


def run_gpu(ctx, batch, budget, mem=True, digest=False):
    h = ctx.load(batch)
    ctx.run(h, budget)
    out = ctx.fetch(h, mem=mem, digest=digest)
    ctx.free(h)
    return out


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_plain_small_bit_exact(ctx, rasp, sched):
    print("case: plain-small sched=%s" % sched, flush=True)
    configure(ctx, rasp, sched)
    b = W.config1()
    compare(run_gpu(ctx, b, b.budget), oracle.run(b, b.budget, threads=4))


@pytest.mark.parametrize("sched", list(SCHEDULES))
@pytest.mark.parametrize("isa", [0, 1])
def test_tiny_ragged_machines_bit_exact(ctx, rasp, sched, isa):
    """Ragged m, n, l, s (n not a multiple of 4, l = 0, s = 0), negative and
    out-of-range operands, opcodes beyond the set, odd jump targets."""
    print("case: tiny-ragged sched=%s isa=%d" % (sched, isa), flush=True)
    configure(ctx, rasp, sched)
    b = W.tiny_random(seed=11 + isa, num_vms=5000, isa=isa, max_m=10, max_n=37,
                      operand_lo=-60, operand_hi=60)
    compare(run_gpu(ctx, b, 300), oracle.run(b, 300))


def _hand_cases():
    with open(os.path.join(GOLDEN, "hand_traces.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("sched", ["plain", "persistent-lds32"])
def test_hand_traced_machines(ctx, rasp, sched):
    configure(ctx, rasp, sched)
    for case in _hand_cases():
        print("case: hand %s sched=%s" % (case["name"], sched), flush=True)
        isa = W.ISA_CLASSIC if case["isa"] == "classic" else W.ISA_WORD
        b = W.from_programs(isa, [case["words"]], case["n"], [case["tape"]],
                            ell=case["ell"], s=case["s"])
        got = run_gpu(ctx, b, case["budget"])
        e = case["expect"]
        assert int(got["steps"][0]) == e["steps"], case["name"]
        assert int(got["status"][0]) == e["halted"], case["name"]
        assert (int(got["i"][0]), int(got["a"][0])) == (e["i"], e["a"]), case["name"]
        assert got["y"].tolist() == e["Y"], case["name"]
        compare(got, oracle.run(b, case["budget"]))


def test_busy_beavers_word_set(ctx, rasp):
    """App. B programs lowered to the word RASP, 32-bit words, on the GPU."""
    configure(ctx, rasp, "persistent-lds32")
    with open(os.path.join(GOLDEN, "busy_beavers.json")) as f:
        spec = json.load(f)
    m = spec["machine"]
    progs = []
    for p in spec["programs"]:
        with open(os.path.join(GOLDEN, p["file"])) as f:
            pairs, _ = dsl.lower_word(dsl.parse(f.read()), ell=m["ell"], s=m["s"], mu=m["mu"])
        progs.append(dsl.flatten(pairs))
    b = W.from_programs(W.ISA_WORD, progs, m["n"], [[]] * 3, ell=m["ell"], s=m["s"])
    got = run_gpu(ctx, b, 10 ** 6)
    want = oracle.run(b, 10 ** 6)
    compare(got, want)
    assert (got["status"] == 1).all()


@pytest.mark.parametrize("sched", ["plain", "firstpass-lds64"])
def test_uneven_batch_reduced_bit_exact(ctx, rasp, sched):
    print("case: uneven N=20000 sched=%s" % sched, flush=True)
    configure(ctx, rasp, sched)
    b = W.config3(num_vms=20000, budget=4096)
    compare(run_gpu(ctx, b, b.budget), oracle.run(b, b.budget, threads=8))


def test_split_budget_and_halted_machines(ctx, rasp):
    configure(ctx, rasp, "firstpass-lds64")
    b = W.config1()
    h = ctx.load(b)
    ctx.run(h, 100)
    ctx.run(h, 156)
    got = ctx.fetch(h, mem=True)
    compare(got, oracle.run(b, 256))
    ctx.run(h, 1000)
    again = ctx.fetch(h, mem=True)
    halted = got["status"] == 1
    for k in ("i", "a", "steps", "u0", "y0"):
        assert np.array_equal(again[k][halted], got[k][halted])
    ctx.free(h)
