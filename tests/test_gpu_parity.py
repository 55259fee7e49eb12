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
# kind 0: the first pass is the plain kernel; kind 1: the persistent kernel
# with memory in LDS (when every memory fits its slot, else the plain kernel)
SCHEDULES = {
    "plain": dict(schedule=1),
    "persistent-hbm": dict(schedule=2, first_pass=0, lds_words=0, epoch=16, kind=1),
    "persistent-lds32": dict(schedule=2, first_pass=0, lds_words=32, epoch=8, kind=1),
    "firstpass-lds64": dict(schedule=2, first_pass=4, lds_words=64, epoch=32, kind=0),
    "firstpass-lds16-tiny-epoch": dict(schedule=2, first_pass=1, lds_words=16, epoch=1, kind=0),
    "ldsfirst-lds64": dict(schedule=2, first_pass=5, lds_words=64, epoch=32, kind=1),
    "ldsfirst-lds1024-epoch3": dict(schedule=2, first_pass=7, lds_words=1024, epoch=3, kind=1),
    # slots of 208 and 160 words: three one-wave blocks, one four-wave block
    # per compute unit; memories above 208 / 156 words are split
    "persistent-lds208-split": dict(schedule=2, first_pass=64, lds_words=208, epoch=64, kind=0),
    "persistent-lds156-split": dict(schedule=2, first_pass=0, lds_words=156, epoch=16, kind=0),
    # hot-cell tables: a profiled plain first pass, then each survivor's
    # profiled cells hashed into S LDS slots (misfits keep what fits)
    "persistent-lds16-split": dict(schedule=2, first_pass=0, lds_words=16, epoch=2, kind=0),
    "hot16": dict(schedule=2, first_pass=64, lds_words=0, epoch=16, kind=0, hot=16, prof=32),
    "hot8-tiny-epoch": dict(schedule=2, first_pass=3, lds_words=0, epoch=1, kind=0, hot=8, prof=2,
                            misfit_waves=1),
    "hot64-long-profile": dict(schedule=2, first_pass=40, lds_words=0, epoch=64, kind=0, hot=64, prof=40),
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


@pytest.fixture(autouse=True)
def no_hot_cells(ctx, rasp):
    """Tests that set knobs themselves start without hot-cell tables."""
    ctx.set(rasp.RASP_OPT_HOT_CELLS, 0)
    ctx.set(rasp.RASP_OPT_PROFILE_STEPS, 256)
    yield


def configure(ctx, rasp, sched):
    o = SCHEDULES[sched]
    ctx.set(rasp.RASP_OPT_SCHEDULE, o["schedule"])
    if "first_pass" in o:
        ctx.set(rasp.RASP_OPT_FIRST_PASS, o["first_pass"])
        ctx.set(rasp.RASP_OPT_LDS_WORDS, o["lds_words"])
        ctx.set(rasp.RASP_OPT_EPOCH, o["epoch"])
        ctx.set(rasp.RASP_OPT_FIRST_PASS_KIND, o["kind"])
    ctx.set(rasp.RASP_OPT_HOT_CELLS, o.get("hot", 0))
    ctx.set(rasp.RASP_OPT_PROFILE_STEPS, o.get("prof", 256))
    ctx.set(rasp.RASP_OPT_MISFIT_WAVES, o.get("misfit_waves", 6))


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


@pytest.mark.parametrize("sched", ["plain", "persistent-hbm", "persistent-lds32", "persistent-lds16-split",
                                   "hot8-tiny-epoch"])
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


@pytest.mark.parametrize("sched", ["plain", "firstpass-lds64", "ldsfirst-lds1024-epoch3", "hot16",
                                   "hot8-tiny-epoch", "hot64-long-profile"])
def test_uneven_batch_reduced_bit_exact(ctx, rasp, sched):
    print("case: uneven N=20000 sched=%s" % sched, flush=True)
    configure(ctx, rasp, sched)
    b = W.config3(num_vms=20000, budget=4096)
    compare(run_gpu(ctx, b, b.budget), oracle.run(b, b.budget, threads=8))


def _image(n, words):
    """A program as a memory image: words[k] at word k (a dict), zeros elsewhere,
    as many words as the highest one set (rounded up to even)."""
    top = max(words) + 1
    img = [0] * (top + (top & 1))
    for k, w in words.items():
        img[k] = w
    assert len(img) <= n
    return img


def _boundary_programs(n):
    """Classic programs that hit the split slot's and the hot-cell table's
    boundary positions at P = 16 LDS words (memory of n > 16 words)."""
    LOAD, ADD, STORE, JPOS, PRINT, JMP = 1, 2, 4, 5, 7, 8
    return [
        # the operand of the instruction at n - 1 wraps to word 0: LOAD M[0]
        _image(n, {0: LOAD, 1: LOAD, 2: STORE, 3: n - 1, 4: JMP, 5: n - 1}),
        # a misaligned instruction at P - 1 whose operand is word P (in HBM)
        _image(n, {0: JMP, 1: 15, 15: LOAD, 16: 77, 17: PRINT, 18: 16}),
        # a store into the next instruction's operand, across P, in a loop
        _image(n, {0: JMP, 1: 12, 12: LOAD, 13: 55, 14: STORE, 15: 17, 16: ADD, 17: 99,
                   18: PRINT, 19: 17, 20: STORE, 21: 15, 22: JPOS, 23: 14}),
        # a store into the opcode word of the instruction at P - 1 just before
        # it is fetched
        _image(n, {0: LOAD, 1: PRINT, 2: STORE, 3: 15, 4: JMP, 5: 15, 16: 2}),
        # a jump to P - 2 and a loop whose data word is its own next opcode
        _image(n, {0: JMP, 1: 14, 14: ADD, 15: 16, 16: STORE, 17: 16, 18: JPOS, 19: 14}),
    ]


@pytest.mark.parametrize("sched", ["plain", "persistent-lds16-split", "firstpass-lds16-tiny-epoch",
                                   "hot8-tiny-epoch", "hot16"])
@pytest.mark.parametrize("n", [41, 64])
def test_split_and_hot_table_boundaries(ctx, rasp, sched, n):
    """Hand-built machines at the split slot's boundary (P = 16 words in LDS,
    the rest in HBM): an operand wrapping from word n - 1 to word 0, a
    misaligned instruction at P - 1 whose operand is word P, stores into the
    next instruction's words just before its fetch on both sides of P; the
    same positions are cell boundaries of the hot-cell tables."""
    print("case: boundaries n=%d sched=%s" % (n, sched), flush=True)
    configure(ctx, rasp, sched)
    progs = _boundary_programs(n)
    b = W.from_programs(W.ISA_CLASSIC, progs, n, [[3, -4]] * len(progs), ell=2, s=2)
    compare(run_gpu(ctx, b, 300), oracle.run(b, 300))


@pytest.fixture(scope="module")
def rollouts_reduced():
    b = W.config4(num_vms=512)
    return b, oracle.run(b, b.budget, threads=8)


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_rollouts_reduced_bit_exact(ctx, rasp, rollouts_reduced, sched):
    """512 distinct counted-loop array programs (n = 2,048, budget 2^20) under
    every schedule: memory slices larger than any slot, long READ and PRINT
    bursts."""
    b, want = rollouts_reduced
    print("case: rollouts N=%d sched=%s" % (b.N, sched), flush=True)
    configure(ctx, rasp, sched)
    compare(run_gpu(ctx, b, b.budget), want)


def test_poll_and_sync_per_batch(ctx, rasp):
    """rasp_poll / rasp_sync on one batch wait for that batch's queued work;
    batch 0 means all work of the context; an unknown handle is an error."""
    configure(ctx, rasp, "firstpass-lds64")
    b = W.config1()
    h1, h2 = ctx.load(b), ctx.load(b)
    ctx.run(h1, 256)
    ctx.run(h2, 100)
    ctx.sync(h1)
    assert ctx.poll(h1)
    ctx.sync(h2)
    assert ctx.poll(h2) and ctx.poll(0)
    ctx.run(h2, 156)
    ctx.sync(0)
    assert ctx.poll(h2)
    want = oracle.run(b, 256)
    compare(ctx.fetch(h1, mem=True), want)
    compare(ctx.fetch(h2, mem=True), want)
    ctx.free(h1)
    with pytest.raises(rasp.RaspError, match="unknown batch handle"):
        ctx.poll(h1)
    with pytest.raises(rasp.RaspError, match="unknown batch handle"):
        ctx.sync(h1)
    ctx.free(h2)


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


def test_run_multi_equals_separate_runs(ctx, rasp):
    """One launch over several batches (different shapes and budgets) equals
    running each batch alone."""
    configure(ctx, rasp, "firstpass-lds64")
    batches = [W.config1(seed=21), W.tiny_random(seed=22, num_vms=3000, max_n=40),
               W.config3(num_vms=3000, seed=23, budget=2000)]
    budgets = [256, 150, 2000]
    hs = [ctx.load(b) for b in batches]
    ctx.run_multi(hs, budgets)
    for h, b, bud in zip(hs, batches, budgets):
        compare(ctx.fetch(h, mem=True), oracle.run(b, bud))
        ctx.free(h)


def _random_states(b, seed):
    """Arbitrary reachable-shaped states: i, a anywhere in int32 (edge values
    included), u0 <= l, y0 <= s, memory words random with edge values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = oracle.init(b)
    N = b.N
    edges = np.array([0, 1, -1, 2, -2, 2 ** 31 - 1, -2 ** 31, 2 ** 31 - 2, -2 ** 31 + 1], np.int64)
    pick = lambda k: np.where(rng.random(k) < 0.3, edges[rng.integers(0, len(edges), k)],
                              rng.integers(-2 ** 31, 2 ** 31, k)).astype(np.int32)
    st.i = np.where(rng.random(N) < 0.5, rng.integers(-4, 40, N), pick(N)).astype(np.int32)
    st.a = pick(N)
    st.u0 = np.floor(rng.random(N) * (st.l.astype(np.int64) + 1)).astype(np.uint32)
    st.y0 = np.floor(rng.random(N) * (st.s.astype(np.int64) + 1)).astype(np.uint32)
    small = rng.integers(-3, 12, st.mem.size).astype(np.int32)
    st.mem = np.where(rng.random(st.mem.size) < 0.2, pick(st.mem.size), small).astype(np.int32)
    st.steps = rng.integers(0, 1000, N).astype(np.uint64)
    st.Y = rng.integers(-9, 9, st.Y.size).astype(np.int32)
    return st


@pytest.mark.parametrize("sched", ["plain", "persistent-hbm", "persistent-lds32", "firstpass-lds16-tiny-epoch",
                                   "ldsfirst-lds64", "hot8-tiny-epoch"])
@pytest.mark.parametrize("isa", [0, 1])
def test_loaded_states_fuzz(ctx, rasp, sched, isa):
    """rasp_load_state with arbitrary configurations (i near INT32_MAX, odd,
    negative; a and memory words at the int32 edges; u0 = l; y0 = s), then 1
    and 37 transitions, against the oracle advanced from the same state."""
    configure(ctx, rasp, sched)
    b = W.tiny_random(seed=40 + isa, num_vms=4000, isa=isa, max_m=6, max_n=30, max_ell=4,
                      max_s=3, opcode_hi=10)
    st = _random_states(b, seed=41 + isa)
    state = dict(i=st.i, a=st.a, u0=st.u0, y0=st.y0, steps=st.steps, y=st.Y, mem=st.mem)
    h = ctx.load_state(b, state)
    got0 = ctx.fetch(h, mem=True)
    want = st.copy()
    oracle.advance(want, 0)
    compare(got0, want)
    for budget in (1, 37):
        ctx.run(h, budget)
        oracle.advance(want, budget)
        compare(ctx.fetch(h, mem=True), want)
    ctx.free(h)


def test_order_and_halves(ctx, rasp):
    """A permuted batch gives permuted results; a batch equals its two halves
    run separately (machines are independent)."""
    configure(ctx, rasp, "firstpass-lds64")
    b = W.config3(num_vms=4000, seed=31, budget=3000)
    full = run_gpu(ctx, b, 3000)
    perm = np.random.Generator(np.random.PCG64(3)).permutation(b.N)
    pg = run_gpu(ctx, b.subset(perm), 3000, mem=False)
    for k in ("status", "steps", "i", "a", "u0", "y0"):
        assert np.array_equal(pg[k], full[k][perm])
    lo = run_gpu(ctx, b.subset(np.arange(2000)), 3000)
    hi = run_gpu(ctx, b.subset(np.arange(2000, 4000)), 3000)
    for k in ("status", "steps", "i", "a", "u0", "y0", "y", "mem"):
        assert np.array_equal(np.concatenate([lo[k], hi[k]]), full[k]), k


def test_zero_tails_across_runs_and_schedules(ctx, rasp):
    """c0's zero tails are left unstored at load: runs that change schedule
    between them (the plain pass reading unstored words as zero and storing
    a tail at its first write there; a persistent launch without a first
    pass, which needs every tail stored first; hot-cell tables; the
    no-allocation entry point) compose to the oracle's result, with digests
    (read through the mark) and memories (tails stored first) equal."""
    b = W.config3(num_vms=3000, seed=37, budget=4000)
    print("case: zero tails across schedules N=%d" % b.N, flush=True)
    h = ctx.load(b)
    done = 0
    for sched, budget, noalloc in (("plain", 40, False), ("persistent-hbm", 150, False),
                                   ("firstpass-lds64", 300, True), ("hot16", 700, False),
                                   ("persistent-lds156-split", 800, False)):
        configure(ctx, rasp, sched)
        if noalloc:
            rasp.rasp_run_noalloc(ctx.handle, h, budget)
        else:
            ctx.run(h, budget)
        done += budget
        want = oracle.run(b, done)
        got = ctx.fetch(h, digest=True, mem=False)
        compare(got, want, mem=False)
        assert np.array_equal(got["y"], want.Y), sched
        assert np.array_equal(got["mem_digest"], oracle.digest(want)), sched
    got = ctx.fetch(h, mem=True, digest=True)
    compare(got, oracle.run(b, done))
    ctx.free(h)


def test_device_descriptor_and_digest(ctx, rasp):
    """A descriptor of device-resident arrays (ragged shapes) loads the same
    c0 as a host one; memory digests equal the oracle's FNV-1a hashes."""
    configure(ctx, rasp, "firstpass-lds64")
    b = W.config3(num_vms=5000, seed=33, budget=1000)
    d = rasp.make_desc(b, ctx.device)
    h = rasp.rasp_load_batch(ctx.handle, d)
    ctx.run(h, 1000)
    got = ctx.fetch(h, mem=True, digest=True)
    ctx.free(h)
    want = oracle.run(b, 1000)
    compare(got, want)
    assert np.array_equal(got["mem_digest"], oracle.digest(want))


def test_error_paths(ctx, rasp):
    R = rasp
    b = W.config1(num_vms=8)
    # program longer than memory -> INVAL, nothing allocated
    bad = W.config1(num_vms=8)
    bad.mem_words = bad.mem_words.copy()
    bad.mem_words[3] = 10
    with pytest.raises(R.RaspError) as e:
        ctx.load(bad)
    assert e.value.code == R.RASP_E_INVAL
    # same check on the device path
    with pytest.raises(R.RaspError) as e:
        R.rasp_load_batch(ctx.handle, R.make_desc(bad, ctx.device))
    assert e.value.code == R.RASP_E_INVAL
    # decreasing offsets
    bad2 = W.config1(num_vms=8)
    bad2.prog_off = bad2.prog_off.copy()
    bad2.prog_off[4] = bad2.prog_off[5] + 1
    with pytest.raises(R.RaspError) as e:
        ctx.load(bad2)
    assert e.value.code == R.RASP_E_INVAL
    # unknown handle, double free
    h = ctx.load(b)
    ctx.free(h)
    with pytest.raises(R.RaspError) as e:
        ctx.free(h)
    assert e.value.code == R.RASP_E_STATE
    with pytest.raises(R.RaspError) as e:
        ctx.run(h, 5)
    assert e.value.code == R.RASP_E_STATE
    # state with u0 > l
    st = oracle.init(b)
    st.u0 = st.u0.copy()
    st.u0[0] = int(st.l[0]) + 1
    with pytest.raises(R.RaspError) as e:
        ctx.load_state(b, dict(i=st.i, a=st.a, u0=st.u0, y0=st.y0, mem=st.mem))
    assert e.value.code == R.RASP_E_INVAL
    # arena too small
    small = R.Context(2 << 20)
    with pytest.raises(R.RaspError) as e:
        small.load(W.config2(num_vms=20000))
    assert e.value.code == R.RASP_E_NOMEM
    small.close()
    # LDS words per slot: -1, 0 or a multiple of 4 up to 1024
    before = ctx.get(R.RASP_OPT_LDS_WORDS)
    for bad_p in (6, 1028, -2):
        with pytest.raises(R.RaspError) as e:
            ctx.set(R.RASP_OPT_LDS_WORDS, bad_p)
        assert e.value.code == R.RASP_E_INVAL
    assert ctx.get(R.RASP_OPT_LDS_WORDS) == before
    # the context still works after all of the above
    compare(run_gpu(ctx, b, 256), oracle.run(b, 256))


def test_budget_zero_reports_fixed_points_of_c0(ctx, rasp):
    configure(ctx, rasp, "plain")
    b = W.config1()
    got = run_gpu(ctx, b, 0)
    compare(got, oracle.run(b, 0))
    assert got["status"].any() and not got["status"].all()


@pytest.mark.parametrize("sched", ["plain", "persistent-lds32", "firstpass-lds64", "auto"])
def test_lazy_descriptor_equals_eager(ctx, rasp, sched):
    """RASP_DESC_LAZY (c0 built inside the first run) gives the same state as
    an eager load, whichever schedule runs it (fused persistent launch when
    memories fit their LDS slots, else c0 packed first)."""
    if sched == "auto":
        ctx.set(rasp.RASP_OPT_SCHEDULE, 0)
        ctx.set(rasp.RASP_OPT_LDS_WORDS, -1)
        ctx.set(rasp.RASP_OPT_EPOCH, 16)
    else:
        configure(ctx, rasp, sched)
    for b in (W.config1(seed=51), W.tiny_random(seed=52, num_vms=3000, max_n=40),
              W.config2(num_vms=5000, seed=53)):
        d = rasp.make_desc(b, ctx.device, lazy=True)
        h = rasp.rasp_load_batch(ctx.handle, d)
        ctx.run(h, 300)
        got = ctx.fetch(h, mem=True)
        ctx.free(h)
        compare(got, oracle.run(b, 300))


def test_lazy_descriptor_without_run_and_in_a_mix(ctx, rasp):
    ctx.set(rasp.RASP_OPT_SCHEDULE, 0)
    ctx.set(rasp.RASP_OPT_LDS_WORDS, -1)
    b1, b2 = W.config1(seed=61), W.config1(seed=62)
    # fetched before any run: c0, status = fixed point of c0
    h = ctx.load(b1, device_desc=True, lazy=True)
    compare(ctx.fetch(h, mem=True), oracle.run(b1, 0))
    ctx.free(h)
    # a lazy batch (budget 0 and 200) next to an eager one in one launch; the
    # lazy descriptors' device arrays stay alive until the run (Context.load
    # keeps them until the batch is freed)
    ha = ctx.load(b1, device_desc=True, lazy=True)
    hb = ctx.load(b2)
    hc = ctx.load(b2, device_desc=True, lazy=True)
    ctx.run_multi([ha, hb, hc], [200, 150, 0])
    compare(ctx.fetch(ha, mem=True), oracle.run(b1, 200))
    compare(ctx.fetch(hb, mem=True), oracle.run(b2, 150))
    compare(ctx.fetch(hc, mem=True), oracle.run(b2, 0))
    for x in (ha, hb, hc):
        ctx.free(x)


@pytest.mark.parametrize("sched", ["plain", "firstpass-lds64"])
def test_graph_replays_match_eager(ctx, rasp, sched):
    """RASP_OPT_GRAPH: the captured launch sequence is replayed several times,
    with eager work and synchronizations between replays; every replay's state
    equals the oracle's state after the same total budget."""
    configure(ctx, rasp, sched)
    ctx.set(rasp.RASP_OPT_GRAPH, 1)
    try:
        b, other = W.config1(seed=71), W.tiny_random(seed=72, num_vms=2000)
        h = ctx.load(b)
        for rep in range(1, 5):
            ctx.run(h, 70)                               # replay (captured on rep 1)
            got = ctx.fetch(h, mem=True)                 # synchronizes
            compare(got, oracle.run(b, 70 * rep))
            ho = ctx.load(other)                         # eager work between replays
            ctx.run(ho, 33 * rep)
            compare(ctx.fetch(ho, mem=True), oracle.run(other, 33 * rep))
            ctx.free(ho)
        ctx.free(h)
    finally:
        ctx.set(rasp.RASP_OPT_GRAPH, 0)


def test_autotune_leaves_the_batch_and_stays_bit_exact(ctx, rasp):
    R = rasp
    b = W.config3(num_vms=6000, seed=81, budget=2000)
    h = ctx.load(b)
    ctx.run(h, 100)
    before = ctx.fetch(h, mem=True)
    chosen = R.rasp_autotune(ctx.handle, h, 1900, max_vms=3000)
    print("autotune chose", chosen, flush=True)
    assert chosen["best_ms"] > 0
    for k in R.AUTOTUNE_KNOBS:
        assert ctx.get({"schedule": R.RASP_OPT_SCHEDULE, "lds_words": R.RASP_OPT_LDS_WORDS,
                        "first_pass": R.RASP_OPT_FIRST_PASS, "epoch": R.RASP_OPT_EPOCH,
                        "waves_per_cu": R.RASP_OPT_WAVES_PER_CU,
                        "first_pass_kind": R.RASP_OPT_FIRST_PASS_KIND, "hot_cells": R.RASP_OPT_HOT_CELLS,
                        "profile_steps": R.RASP_OPT_PROFILE_STEPS,
                        "misfit_waves": R.RASP_OPT_MISFIT_WAVES}[k]) == chosen[k]
    after = ctx.fetch(h, mem=True)
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    ctx.run(h, 1900)
    compare(ctx.fetch(h, mem=True), oracle.run(b, 2000))
    ctx.free(h)
    # restore the defaults for the other tests
    ctx.set(R.RASP_OPT_SCHEDULE, 0)
    ctx.set(R.RASP_OPT_LDS_WORDS, -1)
    ctx.set(R.RASP_OPT_FIRST_PASS, 64)
    ctx.set(R.RASP_OPT_EPOCH, 256)
    ctx.set(R.RASP_OPT_WAVES_PER_CU, 16)
    ctx.set(R.RASP_OPT_FIRST_PASS_KIND, 0)


def test_autotune_on_a_lazy_batch(ctx, rasp):
    """Tuning a lazily loaded batch leaves it lazy: its first real run still
    builds c0 from the descriptor and the result is bit-exact."""
    R = rasp
    b = W.config3(num_vms=5000, seed=82, budget=1500)
    try:
        h = ctx.load(b, device_desc=True, lazy=True)
        chosen = R.rasp_autotune(ctx.handle, h, 1500, max_vms=2500)
        print("autotune (lazy) chose", chosen, flush=True)
        assert chosen["best_ms"] > 0
        ctx.run(h, 1500)
        compare(ctx.fetch(h, mem=True), oracle.run(b, 1500))
        ctx.free(h)
    finally:
        ctx.set(R.RASP_OPT_SCHEDULE, 0)
        ctx.set(R.RASP_OPT_LDS_WORDS, -1)
        ctx.set(R.RASP_OPT_FIRST_PASS, 64)
        ctx.set(R.RASP_OPT_EPOCH, 256)
        ctx.set(R.RASP_OPT_WAVES_PER_CU, 16)
        ctx.set(R.RASP_OPT_FIRST_PASS_KIND, 0)


@pytest.mark.parametrize("sched", ["plain", "persistent-hbm", "firstpass-lds64", "ldsfirst-lds64",
                                   "persistent-lds208-split", "persistent-lds156-split", "hot16",
                                   "hot64-long-profile"])
def test_fig1_programs_bit_exact(ctx, rasp, sched):
    """Word RASP, n = 250 (the general-n path), uniform Sec. 2.2 programs with
    the input-reading prologue, budget 10^6: every machine."""
    print("case: fig1 N=2048 sched=%s" % sched, flush=True)
    configure(ctx, rasp, sched)
    b = W.fig1(num_vms=2048, seed=12)
    compare(run_gpu(ctx, b, b.budget), oracle.run(b, b.budget, threads=16))


def _to_width(b, w):
    """The batch with every program and input word reduced to a w-bit value
    (sign-extended), marked as a w-bit batch."""
    def red(x):
        x = x.astype(np.int64) & ((1 << w) - 1)
        return np.where(x >= 1 << (w - 1), x - (1 << w), x).astype(np.int32)
    b.prog = red(b.prog)
    b.tape = red(b.tape)
    b.word_bits = w
    return b


@pytest.mark.parametrize("sched", ["plain", "persistent-lds32", "persistent-hbm",
                                   "firstpass-lds16-tiny-epoch", "ldsfirst-lds64", "hot8-tiny-epoch"])
@pytest.mark.parametrize("isa", [0, 1])
@pytest.mark.parametrize("w", [3, 5, 8, 16, 29])
def test_narrow_words_bit_exact(ctx, rasp, sched, isa, w):
    """Words of w < 32 bits (Sec. 2.1, W = F_2^w): arithmetic, i + 1 and i + 2
    wrap mod 2^w; tiny ragged machines whose counters and operands reach the
    w-bit edges, memory sizes both below and above 2^w."""
    print("case: narrow words w=%d isa=%d sched=%s" % (w, isa, sched), flush=True)
    configure(ctx, rasp, sched)
    b = _to_width(W.tiny_random(seed=300 + w + 50 * isa, num_vms=3000, isa=isa, max_m=6,
                                max_n=24, operand_lo=-(1 << 12), operand_hi=1 << 12), w)
    compare(run_gpu(ctx, b, 200), oracle.run(b, 200, w=w))


def test_busy_beavers_halting_numbers_on_gpu(ctx, rasp):
    """App. B's captions on the GPU: the three busy beavers halt after
    exactly 1549, 1272 and 1255 transitions at w = 29, and the whole final
    configurations equal the oracle's at w = 29 and w = 32."""
    configure(ctx, rasp, "persistent-lds32")
    with open(os.path.join(GOLDEN, "busy_beavers.json")) as f:
        spec = json.load(f)
    m = spec["machine"]
    progs = []
    for p in spec["programs"]:
        with open(os.path.join(GOLDEN, p["file"])) as f:
            pairs, _ = dsl.lower_word(dsl.parse(f.read()), ell=m["ell"], s=m["s"], mu=m["mu"])
        progs.append(dsl.flatten(pairs))
    for w in (29, 32):
        b = W.from_programs(W.ISA_WORD, progs, m["n"], [[]] * 3, ell=m["ell"], s=m["s"])
        b.word_bits = w
        got = run_gpu(ctx, b, 10 ** 6)
        compare(got, oracle.run(b, 10 ** 6, w=w))
        assert (got["status"] == 1).all()
        if w == 29:
            assert got["steps"].tolist() == [p["tau_h"] for p in spec["programs"]]


def test_narrow_words_reject_wide_values(ctx, rasp):
    R = rasp
    b = _to_width(W.config1(num_vms=16), 8)
    b.prog = b.prog.copy()
    b.prog[5] = 200                             # not an 8-bit word
    with pytest.raises(R.RaspError) as e:
        ctx.load(b)
    assert e.value.code == R.RASP_E_INVAL
    with pytest.raises(R.RaspError) as e:
        R.rasp_load_batch(ctx.handle, R.make_desc(b, ctx.device))
    assert e.value.code == R.RASP_E_INVAL
    ok = _to_width(W.config1(num_vms=16), 8)
    st = oracle.init(ok, w=8)
    st.a = st.a.copy()
    st.a[2] = 1000                              # a state word wider than 8 bits
    with pytest.raises(R.RaspError) as e:
        ctx.load_state(ok, dict(i=st.i, a=st.a, u0=st.u0, y0=st.y0, mem=st.mem))
    assert e.value.code == R.RASP_E_INVAL
    bad_w = W.config1(num_vms=4)
    bad_w.word_bits = 33
    with pytest.raises(R.RaspError) as e:
        ctx.load(bad_w)
    assert e.value.code == R.RASP_E_INVAL
    compare(run_gpu(ctx, ok, 256), oracle.run(ok, 256, w=8))


def test_fetch_into_device_buffers(ctx, rasp):
    """rasp_fetch_outputs with RASP_OUT_DEVICE_PTRS (what the benchmark times)
    gives the same scalars, outputs and memory as the host fetch, field by
    field and with some fields left out."""
    import torch
    R = rasp
    configure(ctx, rasp, "firstpass-lds64")
    b = W.config3(num_vms=3000, seed=91, budget=800)
    h = ctx.load(b)
    ctx.run(h, 800)
    host = ctx.fetch(h, mem=True)
    dev = ctx.device
    N = b.N
    sum_n = int(b.mem_words.astype(np.int64).sum())
    bufs = dict(status=torch.empty(N, dtype=torch.uint8, device=dev),
                steps=torch.empty(N, dtype=torch.int64, device=dev),
                i=torch.empty(N, dtype=torch.int32, device=dev),
                a=torch.empty(N, dtype=torch.int32, device=dev),
                u0=torch.empty(N, dtype=torch.int32, device=dev),
                y0=torch.empty(N, dtype=torch.int32, device=dev),
                y=torch.empty(int(b.out_cap.astype(np.int64).sum()), dtype=torch.int32, device=dev),
                mem=torch.empty(sum_n, dtype=torch.int32, device=dev))
    R.rasp_fetch_outputs_into(ctx.handle, h, bufs, device=True)
    torch.cuda.synchronize()
    for k in ("status", "steps", "i", "a", "u0", "y0", "y", "mem"):
        got = bufs[k].cpu().numpy()
        want = np.asarray(host[k])
        assert np.array_equal(got.view(want.dtype) if got.dtype != want.dtype else got, want), k
    # a subset of fields: the others stay untouched
    part = dict(steps=torch.full((N,), -7, dtype=torch.int64, device=dev),
                a=torch.full((N,), -7, dtype=torch.int32, device=dev))
    R.rasp_fetch_outputs_into(ctx.handle, h, part, device=True)
    torch.cuda.synchronize()
    assert np.array_equal(part["steps"].cpu().numpy().view(np.uint64), np.asarray(host["steps"]))
    assert np.array_equal(part["a"].cpu().numpy(), np.asarray(host["a"]))
    ctx.free(h)


def test_contexts_on_their_own_threads_and_cu_shares(rasp):
    """What the benchmark's batches in flight rely on: four contexts, each on
    its own quarter of the CUs (rasp_create_on_cus) and driven by its own host
    thread, load, run and fetch different batches at the same time, and every
    result is bit-exact."""
    import threading
    R = rasp
    n = 4
    probe = R.Context(64 << 20)
    cus = R.rasp_device_info(probe.handle)["compute_units"]
    probe.close()
    shares = [R.cu_share(k, n, cus) for k in range(n)]
    assert sum(c for _, c in shares) == cus and shares[0][0] == 0
    ctxs = [R.Context(256 << 20, cus=sh) for sh in shares]
    batches = [W.config1(seed=40 + k, num_vms=3000) if k % 2 == 0 else
               W.config3(num_vms=3000, seed=50 + k, budget=3000) for k in range(n)]
    print("case: %d contexts on CU quarters, 3 rounds each" % n, flush=True)
    got, errors = [[] for _ in range(n)], []

    def drive(k):
        try:
            for _ in range(3):
                got[k].append(run_gpu(ctxs[k], batches[k], batches[k].budget))
        except Exception as e:
            errors.append(e)

    threads = [threading.Thread(target=drive, args=(k,)) for k in range(n)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for c in ctxs:
        c.close()
    assert not errors, errors
    for k in range(n):
        want = oracle.run(batches[k], batches[k].budget, threads=4)
        for out in got[k]:
            compare(out, want)


def test_create_on_cus_rejects_ranges_outside_the_device(rasp):
    R = rasp
    probe = R.Context(64 << 20)
    cus = R.rasp_device_info(probe.handle)["compute_units"]
    probe.close()
    for first, count in ((0, 0), (cus, 1), (cus - 4, 8)):
        with pytest.raises(R.RaspError) as e:
            R.rasp_create_on_cus(0, None, 64 << 20, first, count)
        assert e.value.code == R.RASP_E_INVAL
