"""The Sec. 2.2 grammar sampler and the Sec. 3 workload built on it.

Counts are checked against brute-force enumeration of the grammar, samples
against the counts, and the lowered programs (with the input-reading prologue)
against direct evaluation of the same programs.
"""
import collections
import random

import numpy as np

import oracle
from oracle import dsl_eval
from paper_2604_12902_amd import dsl, grammar, workloads as W

# The Sec. 2.2 grammar written out as data, for a brute-force enumerator that
# shares nothing with the sampler's counting code.
_RULES = {
    "B": [["S"], ["S", ";", "B"], ["hlt"]],
    "S": [["P", "=", "E"], ["ife", "G", "{", "B", "}", "{", "B", "}"], ["whl", "G", "{", "B", "}"]],
    "Z": [["0"]] + [[d] for d in "123456789"],
    "G": [[a, "[", "Z", "]"] for a in ("ipt", "scr", "opt")],
    "P": [[a, "[", "Z", "]"] for a in ("scr", "opt")],
    "E": [["G", "+", "G"], ["G", "*", "G"], ["G", "+", "Z"], ["G", "*", "Z"], ["G"], ["Z"]],
}


def _enumerate(sym, k, memo):
    """Every terminal string of exactly k symbols derived from `sym`."""
    if sym not in _RULES:
        return [(sym,)] if k == 1 else []
    key = (sym, k)
    if key in memo:
        return memo[key]
    out = []
    for rhs in _RULES[sym]:
        def expand(i, left):
            if i == len(rhs):
                if left == 0:
                    yield ()
                return
            rest_min = len(rhs) - i - 1             # every symbol yields >= 1 terminal
            for take in range(1, left - rest_min + 1):
                for head in _enumerate(rhs[i], take, memo):
                    for tail in expand(i + 1, left - take):
                        yield head + tail
        out.extend(expand(0, k))
    memo[key] = out
    return out


def test_counts_equal_brute_force_enumeration():
    memo = {}
    for k in range(1, 16):
        strings = _enumerate("B", k, memo)
        assert len(strings) == len(set(strings)), "grammar ambiguous at length %d" % k
        assert grammar.count_B(k) == len(strings), k
        assert grammar.count_S(k) == len(_enumerate("S", k, memo)), k


def test_samples_have_exact_length_parse_and_round_trip():
    rng = random.Random(1)
    for L in (16, 21, 40, 100, 120):
        for _ in range(50):
            src = grammar.sample_program(L, rng)
            toks = src.split()
            assert len(toks) == L
            assert dsl.tokenize(src) == toks
            dsl.parse(src)


def test_sampler_is_uniform_on_a_small_length():
    """B of 6 terminals: the 200 assignments ``P = Z``; L = 21 programs are the
    81 x 200 of them.  Chi-square of 40,000 draws over the 200 bodies."""
    assert grammar.count_B(6) == 200 and grammar.count_F(21) == 81 * 200
    rng = random.Random(7)
    counts = collections.Counter(" ".join(grammar.sample_program(21, rng).split()[14:20])
                                 for _ in range(40000))
    assert len(counts) == 200
    obs = np.array(list(counts.values()), dtype=float)
    chi2 = ((obs - 200.0) ** 2 / 200.0).sum()
    assert chi2 < 290                       # 199 dof: P(chi2 > 290) < 1e-4


def test_sampler_production_frequencies_follow_the_counts():
    """For B of 30 terminals: the share of bodies that are a single statement
    equals count_S(30) / count_B(30)."""
    rng = random.Random(3)
    single = 0
    draws = 6000
    for _ in range(draws):
        toks = grammar.sample_program(45, rng).split()[14:-1]
        depth, top_semis = 0, 0
        for t in toks:
            depth += t == "{"
            depth -= t == "}"
            top_semis += (t == ";") and depth == 0
        single += top_semis == 0 and toks != ["hlt"]
    p = grammar.count_S(30) / grammar.count_B(30)
    sd = (p * (1 - p) / draws) ** 0.5
    assert abs(single / draws - p) < 5 * sd


def test_fig1_workload_fits_and_is_seeded():
    a = W.fig1(num_vms=300)
    b = W.fig1(num_vms=300)
    assert a.sha256() == b.sha256()
    assert W.fig1(num_vms=300, seed=6).sha256() != a.sha256()
    assert (a.mem_words == 250).all() and (a.tape_cap == 10).all() and (a.out_cap == 2).all()
    two_m = np.diff(a.prog_off.astype(np.int64))
    assert (two_m + 27 <= 250).all()
    arity = np.diff(a.tape_off.astype(np.int64))
    assert arity.min() >= 1 and arity.max() <= 9
    # program v of a larger batch is the same program
    c = W.fig1(num_vms=310)
    assert np.array_equal(c.prog[:a.prog.size], a.prog)


def test_fig1_programs_print_what_direct_evaluation_prints():
    """Lowered with the READ prologue and run on the oracle, every program
    that halts prints exactly the opt words that evaluating its source on the
    same input gives (w = 32, l = 10, s = 2, mu = 10)."""
    N = 400
    b = W.fig1(num_vms=N, seed=9)
    st = oracle.run(b, 100000)                  # > 12 transitions per evaluated statement
    halted = 0
    for v in range(N):
        fun = dsl.parse(W.fig1_source(9, v))
        x = b.tape[int(b.tape_off[v]):int(b.tape_off[v + 1])].tolist()
        try:
            want = dsl_eval.eval_paper(fun, w=32, ipt=x, mu=10, s=2, ell=10, fuel=5000)
        except dsl_eval.OutOfFuel:
            assert st.steps[v] >= 5000, v           # at least one transition per statement
            continue
        assert st.status[v] == 1, v
        halted += 1
        assert st.out_of(v)[:int(st.y0[v])].tolist() == want, v
    assert halted > N // 2
