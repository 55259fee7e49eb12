"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: the expected values come
from hand traces of the Sec. 1.1 / Sec. 2.1 case tables, the halting numbers
printed in App. B, the definitional whole-vector form of the transition, an
independent unbounded-integer interpreter, a direct evaluator of the array
language, and invariants that every run must satisfy.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import dsl_eval, zinterp
from paper_2604_12902_amd import dsl, workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ISA = {"classic": oracle.ISA_CLASSIC, "word": oracle.ISA_WORD}


def _hand_cases():
    with open(os.path.join(GOLDEN, "hand_traces.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["name"])
def test_hand_traced_machines(case):
    b = W.from_programs(ISA[case["isa"]], [case["words"]], case["n"], [case["tape"]],
                        ell=case["ell"], s=case["s"])
    st = oracle.run(b, case["budget"])
    e = case["expect"]
    assert int(st.steps[0]) == e["steps"]
    assert int(st.status[0]) == e["halted"]
    assert int(st.i[0]) == e["i"]
    assert int(st.a[0]) == e["a"]
    assert int(st.u0[0]) == e["u0"]
    assert int(st.y0[0]) == e["y0"]
    assert st.out_of(0).tolist() == e["Y"]
    mem = np.zeros(case["n"], np.int64)
    mem[:len(case["words"])] = case["words"]
    for k, v in e["mem"].items():
        mem[int(k)] = v
    assert st.mem_of(0).astype(np.int64).tolist() == mem.tolist()


def _busy_beavers():
    with open(os.path.join(GOLDEN, "busy_beavers.json")) as f:
        spec = json.load(f)
    out = []
    for p in spec["programs"]:
        with open(os.path.join(GOLDEN, p["file"])) as f:
            out.append((p["file"], f.read(), p["tau_h"]))
    return spec["machine"], out


def _bb_batch(src, mach):
    pairs, lay = dsl.lower_word(dsl.parse(src), ell=mach["ell"], s=mach["s"], mu=mach["mu"])
    assert 2 * len(pairs) + lay.data_words <= mach["n"]
    return W.from_programs(W.ISA_WORD, [dsl.flatten(pairs)], mach["n"], [[]],
                           ell=mach["ell"], s=mach["s"])


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_busy_beaver_halting_numbers(idx):
    """App. B prints tau_h for BB #1..#3; they come out exactly at w = 29."""
    mach, progs = _busy_beavers()
    name, src, tau = progs[idx]
    st = oracle.run(_bb_batch(src, mach), 10 ** 6, w=29)
    assert int(st.status[0]) == oracle.HALTED
    assert int(st.steps[0]) == tau, name
    assert int(st.y0[0]) == 1 and st.out_of(0).tolist() == [0, 0]


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_busy_beaver_tau_affine_in_word_width(idx):
    """Each loop of the beavers ends by wraparound after w-2, w-1 or w trips,
    so tau_h(w) has a constant difference in w (closed-form trip counts)."""
    mach, progs = _busy_beavers()
    _, src, tau = progs[idx]
    b = _bb_batch(src, mach)
    taus = {w: int(oracle.run(b, 10 ** 6, w=w).steps[0]) for w in range(20, 33)}
    diffs = {taus[w] - taus[w - 1] for w in range(21, 33)}
    assert len(diffs) == 1 and diffs.pop() > 0
    assert taus[29] == tau


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_busy_beaver_output_matches_direct_evaluation(idx):
    mach, progs = _busy_beavers()
    _, src, _ = progs[idx]
    fun = dsl.parse(src)
    for w in (29, 32):
        st = oracle.run(_bb_batch(src, mach), 10 ** 6, w=w)
        want = dsl_eval.eval_paper(fun, w=w, mu=mach["mu"], s=mach["s"])
        assert st.out_of(0)[:int(st.y0[0])].tolist() == want


@pytest.mark.parametrize("isa", [oracle.ISA_CLASSIC, oracle.ISA_WORD])
@pytest.mark.parametrize("w", [3, 5, 8, 32])
def test_interpreter_equals_whole_vector_definition(isa, w):
    """Brute force on tiny machines: the in-place interpreter against Phi_w
    applied to the whole configuration vector, with F = {c : Phi_w(c) = c}."""
    b = W.tiny_random(seed=100 + w + 7 * isa, num_vms=300, isa=isa,
                      operand_lo=-(1 << (w - 1)) if w < 8 else -40,
                      operand_hi=(1 << (w - 1)) - 1 if w < 8 else 40)
    c0 = oracle.init(b, w=w)
    st = c0.copy()
    oracle.advance(st, 40)
    for v in range(b.N):
        n, l, s = int(st.n[v]), int(st.l[v]), int(st.s[v])
        fin, t, halted = oracle.run_literal(isa, w, n, l, s, oracle.vector_of(c0, v), 40)
        assert t == int(st.steps[v]), v
        assert halted == bool(st.status[v]), v
        assert fin.tolist() == oracle.vector_of(st, v).tolist(), v


def test_unbounded_integer_interpreter_agrees_where_nothing_overflows():
    b = W.tiny_random(seed=7, num_vms=2000, max_m=8, max_n=24, operand_lo=-300,
                      operand_hi=300)
    st = oracle.run(b, 200)
    agree = overflow = 0
    for v in range(b.N):
        prog = b.prog[int(b.prog_off[v]):int(b.prog_off[v + 1])].tolist()
        tape = b.tape[int(b.tape_off[v]):int(b.tape_off[v + 1])].tolist()
        z = zinterp.zrun(b.isa, prog, tape, int(b.mem_words[v]), int(b.tape_cap[v]),
                         int(b.out_cap[v]), 200)
        if z["overflow"]:
            overflow += 1
            continue
        assert z["steps"] == int(st.steps[v]) and z["halted"] == bool(st.status[v])
        assert (z["i"], z["a"], z["u0"], z["y0"]) == (int(st.i[v]), int(st.a[v]),
                                                     int(st.u0[v]), int(st.y0[v]))
        assert z["M"] == st.mem_of(v).tolist() and z["Y"] == st.out_of(v).tolist()
        agree += 1
    assert agree > 1900


def test_unbounded_integer_interpreter_sees_wraparound():
    """A doubling loop leaves int32: Z keeps growing, the word machine wraps."""
    words = [1, 1, 4, 20, 1, 0, 2, 20, 2, 20, 4, 20, 8, 4]   # M20=1; loop: a=2*M20; M20=a
    b = W.from_programs(W.ISA_CLASSIC, [words], 24, [[]], s=1)
    st = oracle.run(b, 200)
    z = zinterp.zrun(W.ISA_CLASSIC, words, [], 24, 0, 1, 200)
    assert z["overflow"]
    assert z["M"][20] != int(st.mem_of(0)[20])
    assert z["M"][20] % (1 << 32) == int(st.mem_of(0)[20]) % (1 << 32)


def test_rollout_programs_match_direct_evaluation_and_never_overflow():
    b = W.config4(num_vms=6, num_distinct=6)
    st = oracle.run(b, b.budget)
    for v in range(b.N):
        assert int(st.status[v]) == oracle.HALTED
        tape = b.tape[int(b.tape_off[v]):int(b.tape_off[v + 1])].tolist()
        want = dsl_eval.eval_counted(W.rollout_program(3, v), tape, int(b.out_cap[v]))
        assert st.out_of(v)[:int(st.y0[v])].tolist() == want


@pytest.mark.parametrize("part", range(4))
def test_rollout_population_never_leaves_int32(part):
    """The first 256 machines of the full rollout population (machine v of a
    smaller batch is machine v of the full one: programs come from (seed, v)
    streams and tapes row by row), run over unbounded integers: no value ever
    leaves int32, and the Z machine retires the same steps and prints the same
    words as the int32 oracle."""
    b = W.config4(num_vms=256)
    lo, hi = 64 * part, 64 * (part + 1)
    st = oracle.run(b.subset(np.arange(lo, hi)), b.budget)
    for v in range(lo, hi):
        prog = b.prog[int(b.prog_off[v]):int(b.prog_off[v + 1])].tolist()
        tape = b.tape[int(b.tape_off[v]):int(b.tape_off[v + 1])].tolist()
        z = zinterp.zrun(b.isa, prog, tape, W.ROLLOUT_MEM, W.ROLLOUT_ARRAY, W.ROLLOUT_OUT,
                         b.budget)
        assert not z["overflow"], v
        assert z["steps"] == int(st.steps[v - lo]) and z["Y"] == st.out_of(v - lo).tolist(), v


# ---- invariants on a random batch (the plain small workload) ------------------------

@pytest.fixture(scope="module")
def small():
    b = W.config1()
    return b, oracle.run(b, b.budget, threads=4)


def test_split_budget_composes(small):
    b, full = small
    st = oracle.init(b)
    oracle.advance(st, 100)
    oracle.advance(st, b.budget - 100)
    for k in ("i", "a", "u0", "y0", "steps", "status", "mem", "Y"):
        assert np.array_equal(getattr(st, k), getattr(full, k)), k


def test_halted_machines_never_change(small):
    b, full = small
    st = full.copy()
    oracle.advance(st, 1000)
    h = full.status == oracle.HALTED
    assert h.any()
    for k in ("i", "a", "u0", "y0", "steps"):
        assert np.array_equal(getattr(st, k)[h], getattr(full, k)[h]), k
    for v in np.flatnonzero(h)[:500]:
        assert np.array_equal(st.mem_of(v), full.mem_of(v))


def test_machine_order_does_not_matter(small):
    b, full = small
    perm = np.random.Generator(np.random.PCG64(5)).permutation(b.N)
    st = oracle.run(b.subset(perm), b.budget)
    sub = oracle.subset(full, perm)
    for k in ("i", "a", "u0", "y0", "steps", "status", "mem", "Y"):
        assert np.array_equal(getattr(st, k), getattr(sub, k)), k


def test_output_count_equals_print_steps_and_counters_stay_in_range(small):
    """Step one transition at a time and count executed PRINTs and READs; with
    s = budget the output count equals the PRINT count and u0 the READ count."""
    b, full = small
    st = oracle.init(b)
    prints = np.zeros(b.N, np.int64)
    reads = np.zeros(b.N, np.int64)
    for _ in range(b.budget):
        before = st.steps.copy()
        ops = np.array([st.mem_of(v)[int(st.i[v]) % int(st.n[v])] for v in range(b.N)])
        oracle.advance(st, 1)
        moved = st.steps != before
        prints += moved & (ops == W.PRINT)
        reads += moved & (ops == W.READ)
    assert np.array_equal(st.steps, full.steps)
    assert np.array_equal(full.y0.astype(np.int64), np.minimum(prints, full.s))
    assert np.array_equal(full.u0.astype(np.int64), reads)
    assert (full.u0 <= full.l).all() and (full.steps <= b.budget).all()
    for v in range(b.N):
        assert not full.out_of(v)[int(full.y0[v]):].any()


def test_threads_do_not_change_results(small):
    b, full = small
    st = oracle.run(b, b.budget, threads=1)
    for k in ("i", "a", "u0", "y0", "steps", "status", "mem", "Y"):
        assert np.array_equal(getattr(st, k), getattr(full, k)), k


def test_fnv1a64_published_vectors():
    # offset basis = hash of the empty string (Fowler/Noll/Vo reference values)
    assert oracle.fnv1a64(np.zeros(0, np.int32)) == 0xcbf29ce484222325
    # the word 0x61 hashes its little-endian bytes 61 00 00 00; FNV-1a of "a"
    # is 0xaf63dc4c8601ec8c, then three zero bytes each multiply by the prime
    h = 0xaf63dc4c8601ec8c
    for _ in range(3):
        h = (h * 0x100000001b3) % (1 << 64)
    assert oracle.fnv1a64(np.array([0x61], np.int32)) == h
