"""Seeded synthetic workloads: batches of RASP programs and input tapes.

This module produces inputs only.  It holds none of the step semantics and is
the one piece of code that the GPU path and the CPU oracle both consume.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` in a fixed,
documented order, so a (config, seed, size) triple always yields the same bytes
(``Batch.sha256`` fingerprints them).

Opcode numbers of the classic instruction set (Sec. 1.1 numbering, JMP added):
HALT 0, LOAD 1, ADD 2, SUB 3, STORE 4, JPOS 5, READ 6, PRINT 7, JMP 8.
A program of m instructions is the 2m words (opcode, operand)*, stored at
memory words 0..2m of its machine (the stored-program machine of Sec. 1/2).

Integer ranges written [a, b] are inclusive, [a, b) half-open.  A log-uniform
integer on [a, b] is floor(exp(U(ln a, ln(b + 1)))), clipped to b.
"""
from __future__ import annotations

import hashlib
import math
import random
from dataclasses import dataclass, field

import numpy as np

from . import dsl, grammar

ISA_WORD = 0
ISA_CLASSIC = 1

HALT, LOAD, ADD, SUB, STORE, JPOS, READ, PRINT, JMP = 0, 1, 2, 3, 4, 5, 6, 7, 8
CLASSIC_NAMES = {HALT: "HALT", LOAD: "LOAD", ADD: "ADD", SUB: "SUB", STORE: "STORE",
                 JPOS: "JPOS", READ: "READ", PRINT: "PRINT", JMP: "JMP"}


@dataclass
class Batch:
    """A batch of machines in packed form (what ``rasp_load_batch`` takes).

    prog      int32[sum 2m]   program words, machine v at prog[prog_off[v]:prog_off[v+1]]
    prog_off  uint64[N+1]
    mem_words uint32[N]       memory size n_v (>= 2 m_v)
    tape      int32[sum |x|]  input words, machine v at tape[tape_off[v]:tape_off[v+1]]
    tape_off  uint64[N+1]
    tape_cap  uint32[N]       tape capacity l_v (>= |x_v|)
    out_cap   uint32[N]       output capacity s_v
    """
    isa: int
    prog: np.ndarray
    prog_off: np.ndarray
    mem_words: np.ndarray
    tape: np.ndarray
    tape_off: np.ndarray
    tape_cap: np.ndarray
    out_cap: np.ndarray
    budget: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)
    word_bits: int = 32               # w of Sec. 2.1: words are w-bit, sign-extended

    @property
    def N(self) -> int:
        return len(self.prog_off) - 1

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.isa).tobytes())
        if self.word_bits != 32:
            h.update(np.int64(self.word_bits).tobytes())
        for arr in (self.prog, self.prog_off, self.mem_words, self.tape,
                    self.tape_off, self.tape_cap, self.out_cap):
            h.update(np.ascontiguousarray(arr).tobytes())
        return h.hexdigest()

    def subset(self, idx) -> "Batch":
        """Machines `idx` (in that order) as a batch of their own."""
        idx = np.asarray(idx, dtype=np.int64)
        po, to = self.prog_off.astype(np.int64), self.tape_off.astype(np.int64)
        plen, tlen = po[idx + 1] - po[idx], to[idx + 1] - to[idx]
        prog = _gather_ranges(self.prog, po[idx], plen)
        tape = _gather_ranges(self.tape, to[idx], tlen)
        return Batch(self.isa, prog, _offsets(plen), self.mem_words[idx].copy(),
                     tape, _offsets(tlen), self.tape_cap[idx].copy(),
                     self.out_cap[idx].copy(), self.budget, self.name + "[subset]",
                     dict(self.meta), self.word_bits)

    def footprint_words(self) -> int:
        return int(self.mem_words.astype(np.int64).sum() + self.tape_cap.astype(np.int64).sum()
                   + self.out_cap.astype(np.int64).sum())


def _offsets(sizes) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(np.asarray(sizes, dtype=np.uint64), out=off[1:])
    return off


def _gather_ranges(arr, starts, lens) -> np.ndarray:
    starts = np.asarray(starts, np.int64)
    lens = np.asarray(lens, np.int64)
    total = int(lens.sum())
    if total == 0:
        return arr[:0].copy()
    rel = np.arange(total, dtype=np.int64) - np.repeat(np.cumsum(lens) - lens, lens)
    return arr[np.repeat(starts, lens) + rel].copy()


def log_uniform_int(rng, a, b, size):
    v = np.floor(np.exp(rng.uniform(math.log(a), math.log(b + 1), size=size))).astype(np.int64)
    return np.clip(v, a, b)


def _uniform_batch(N, m, opcodes_hi, operand_hi, n, ell, tape_lo, tape_hi, s, seed,
                   budget, name):
    """Programs of m instructions, opcodes uniform over the 9 classic names,
    operands uniform on [0, operand_hi), tape words uniform on [tape_lo, tape_hi].
    Draw order: opcodes (N x m), operands (N x m), tapes (N x ell)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops = rng.integers(0, opcodes_hi, size=(N, m), dtype=np.int32)
    opd = rng.integers(0, operand_hi, size=(N, m), dtype=np.int32)
    tape = rng.integers(tape_lo, tape_hi + 1, size=(N, ell), dtype=np.int32)
    prog = np.empty((N, 2 * m), dtype=np.int32)
    prog[:, 0::2] = ops
    prog[:, 1::2] = opd
    return Batch(ISA_CLASSIC, prog.reshape(-1),
                 np.arange(N + 1, dtype=np.uint64) * np.uint64(2 * m),
                 np.full(N, n, np.uint32), tape.reshape(-1),
                 np.arange(N + 1, dtype=np.uint64) * np.uint64(ell),
                 np.full(N, ell, np.uint32), np.full(N, s, np.uint32),
                 budget=budget, name=name,
                 meta=dict(seed=seed, m=m, n=n, ell=ell, s=s))


def config1(seed: int = 0, num_vms: int = 4096) -> Batch:
    """Plain method, small: 4,096 random programs of 16 instructions, operands
    on [0, 32), n = 32 zero-initialised words beyond the program (here n = 2m),
    tape of 8 words on [-8, 8], output capacity 256, budget 256."""
    return _uniform_batch(num_vms, 16, 9, 32, 32, 8, -8, 8, 256, seed, 256,
                          "plain-small 4096x16 n=32 budget=256")


def config2(seed: int = 1, num_vms: int = 1 << 20) -> Batch:
    """Plain kernel at scale: 1,048,576 random programs of 64 instructions,
    operands on [0, 256), n = 256, tape of 32 words on [-100, 100], output
    capacity 16, budget 4,096."""
    return _uniform_batch(num_vms, 64, 9, 256, 256, 32, -100, 100, 16, seed, 4096,
                          "plain-scale 1Mx64 n=256 budget=4096")


def config3(seed: int = 2, num_vms: int = 1 << 22, budget: int = 65536) -> Batch:
    """Uneven batch: lengths L log-uniform on [8, 512]; exactly one HALT at a
    uniform slot, the other slots uniform over the 8 other opcodes; a jump at
    slot k targets an instruction drawn uniformly from [0, k] with probability
    0.15 (backward), else from (k, L] (forward), as a word address 2*target;
    memory n log-uniform on [64, 1024] then raised to 2L; data operands on
    [0, n); tape of 32 words on [-100, 100]; output capacity 16.

    Draw order: L (N), n (N), halt slot (N); then, for each chunk of 2^18
    machines in order: opcodes, backward flags, jump uniforms, data uniforms
    (one per instruction of the chunk); finally the tapes (N x 32).
    """
    N = num_vms
    rng = np.random.Generator(np.random.PCG64(seed))
    L = log_uniform_int(rng, 8, 512, N)
    n = np.maximum(log_uniform_int(rng, 64, 1024, N), 2 * L)
    halt_slot = np.floor(rng.random(N) * L).astype(np.int64)
    prog_off = _offsets(2 * L)
    prog = np.empty(int(prog_off[-1]), dtype=np.int32)
    chunk = 1 << 18
    for c0 in range(0, N, chunk):
        c1 = min(N, c0 + chunk)
        Lc = L[c0:c1]
        tot = int(Lc.sum())
        starts = np.cumsum(Lc) - Lc
        vm = np.repeat(np.arange(c1 - c0, dtype=np.int64), Lc)
        k = np.arange(tot, dtype=np.int64) - np.repeat(starts, Lc)
        ops = rng.integers(1, 9, size=tot, dtype=np.int32)          # 8 non-HALT opcodes
        ops[starts + halt_slot[c0:c1]] = HALT
        back = rng.random(tot, dtype=np.float32) < 0.15
        uj = rng.random(tot)
        ud = rng.random(tot)
        Lv = Lc[vm]
        tgt = np.where(back, np.floor(uj * (k + 1)),                  # [0, k]
                       k + 1 + np.floor(uj * (Lv - k))).astype(np.int64)   # (k, L]
        del Lv, uj
        data = np.floor(ud * n[c0:c1][vm]).astype(np.int64)         # [0, n)
        del ud, vm, k
        is_jump = (ops == JMP) | (ops == JPOS)
        opd = np.where(is_jump, 2 * tgt, data)
        opd[ops == HALT] = 0
        base = int(prog_off[c0])
        prog[base:base + 2 * tot:2] = ops
        prog[base + 1:base + 2 * tot:2] = opd
    tape = rng.integers(-100, 101, size=(N, 32), dtype=np.int32)
    return Batch(ISA_CLASSIC, prog, prog_off, n.astype(np.uint32),
                 tape.reshape(-1), np.arange(N + 1, dtype=np.uint64) * np.uint64(32),
                 np.full(N, 32, np.uint32), np.full(N, 16, np.uint32),
                 budget=budget, name="uneven 4Mx[8,512] n=[64,1024] budget=65536",
                 meta=dict(seed=seed))


def tiny_random(seed: int, num_vms: int, max_m: int = 6, max_n: int = 16,
                max_ell: int = 4, max_s: int = 3, isa: int = ISA_CLASSIC,
                operand_lo: int = -40, operand_hi: int = 40, opcode_hi: int = 10) -> Batch:
    """Tiny random machines for exhaustive comparisons: ragged m, n, l, s,
    negative and out-of-range operands, opcodes beyond the instruction set."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.integers(1, max_m + 1, size=num_vms)
    n = np.maximum(rng.integers(1, max_n + 1, size=num_vms), 2 * m)
    ell = rng.integers(0, max_ell + 1, size=num_vms)
    xl = np.floor(rng.random(num_vms) * (ell + 1)).astype(np.int64)
    s = rng.integers(0, max_s + 1, size=num_vms)
    tot = int(m.sum())
    ops = rng.integers(0, opcode_hi, size=tot)
    opd = rng.integers(operand_lo, operand_hi + 1, size=tot)
    prog = np.empty(2 * tot, dtype=np.int32)
    prog[0::2] = ops
    prog[1::2] = opd
    tape = rng.integers(-50, 51, size=int(xl.sum())).astype(np.int32)
    return Batch(isa, prog, _offsets(2 * m), n.astype(np.uint32), tape, _offsets(xl),
                 ell.astype(np.uint32), s.astype(np.uint32), budget=64,
                 name="tiny-random", meta=dict(seed=seed))


def from_programs(isa, programs, n, tapes=None, ell=None, s=2, budget=0, name="custom") -> Batch:
    """A batch from explicit word lists (programs[v] = [op, opd, op, opd, ...])."""
    N = len(programs)
    tapes = tapes if tapes is not None else [[] for _ in range(N)]
    nn = np.broadcast_to(np.asarray(n, dtype=np.uint32), (N,)).copy()
    plen = np.array([len(p) for p in programs], dtype=np.int64)
    tlen = np.array([len(t) for t in tapes], dtype=np.int64)
    ll = tlen.astype(np.uint32) if ell is None else np.broadcast_to(
        np.asarray(ell, dtype=np.uint32), (N,)).copy()
    ss = np.broadcast_to(np.asarray(s, dtype=np.uint32), (N,)).copy()
    prog = np.array([w for p in programs for w in p], dtype=np.int64).astype(np.int32)
    tape = np.array([w for t in tapes for w in t], dtype=np.int64).astype(np.int32)
    return Batch(isa, prog, _offsets(plen), nn, tape, _offsets(tlen), ll, ss,
                 budget=budget, name=name)


# ---- array-program rollouts (counted loops over an input array) --------------------

ROLLOUT_ARRAY = 1024
ROLLOUT_MEM = 2048
ROLLOUT_OUT = 1024
ROLLOUT_BUDGET = 1 << 20
ROLLOUT_BOUND = 1 << 30          # every value stays below this in magnitude


def _rollout_ast(rng, target_instrs, x_bound=1 << 15):
    """One counted-loop program whose lowering has about `target_instrs`
    instructions.  Static bound: each pass runs len iterations; along any path
    through a body at most P statements change an accumulator, each by at most
    x_bound + 9 beyond the largest accumulator, so after `passes` passes every
    value is below passes * len * P * (x_bound + 9) + x_bound, kept < 2^30."""
    n_acc = int(rng.integers(2, 6))
    passes_n = int(rng.integers(1, 4))
    per_path = max(1, (ROLLOUT_BOUND - x_bound) // (passes_n * ROLLOUT_ARRAY * (x_bound + 9)))

    def operand():
        r = rng.random()
        if r < 0.5:
            return ("x",)
        if r < 0.85:
            return ("k", int(rng.integers(1, 10)))
        return ("z",)

    def cond():
        r = rng.random()
        if r < 0.5:
            return ("x",)
        if r < 0.75:
            return ("acc", int(rng.integers(0, n_acc)))
        return ("diff", int(rng.integers(0, n_acc)))

    def stmt_cost(st):                 # instructions emitted by the lowering
        if st[0] == "acc":
            return {"z": 3, "x": 4, "k": 6}[st[4][0]]
        if st[0] == "print":
            return 1
        c = {"x": 2, "acc": 2, "diff": 3}[st[1][0]]
        return c + 2 + sum(stmt_cost(s) for s in st[2]) + sum(stmt_cost(s) for s in st[3])

    def block(budget_instrs, depth, path_left):
        out, used, path = [], 0, 0
        while used < budget_instrs and path < path_left:
            r = rng.random()
            if depth < 3 and r < 0.3 and path_left - path >= 2:
                share = max(4, (budget_instrs - used) // 2)
                then_b, _, tp = block(share // 2, depth + 1, path_left - path)
                else_b, _, ep = block(share // 2, depth + 1, path_left - path)
                st = ("if", cond(), then_b, else_b)
                path += max(tp, ep)
            elif r < 0.36:
                st = ("print", int(rng.integers(0, n_acc)))
            else:
                sign = 1 if rng.random() < 0.5 else -1
                st = ("acc", int(rng.integers(0, n_acc)), int(rng.integers(0, n_acc)),
                      sign, operand())
                path += 1
            out.append(st)
            used += stmt_cost(st)
        return tuple(out), used, path

    fixed = 2 + 14 + passes_n * (17 + n_acc) + 1     # prologue, load loop, pass loops, halt
    body_budget = max(8, (target_instrs - fixed) // passes_n)
    passes = tuple(("pass", block(body_budget, 0, per_path)[0]) for _ in range(passes_n))
    return ("prog", n_acc, ROLLOUT_ARRAY, passes, True)


def rollout_program(seed: int, index: int):
    """AST of rollout program `index` of the family `seed` (independent of N).
    Drawn again (same stream) until its lowering has 128 to 384 instructions."""
    rng = np.random.Generator(np.random.PCG64([seed, index]))
    while True:
        target = int(rng.integers(128, 385))
        ast = _rollout_ast(rng, target)
        if 128 <= len(dsl.lower_classic(ast)[0]) <= 384:
            return ast


def _rollout_chunk(job):
    seed, start, stop = job
    progs = []
    for d in range(start, stop):
        pairs, data_words = dsl.lower_classic(rollout_program(seed, d))
        if 2 * len(pairs) + data_words > ROLLOUT_MEM:
            raise RuntimeError("rollout program does not fit its memory")
        progs.append(np.array(dsl.flatten(pairs), dtype=np.int32))
    return progs


def config4(seed: int = 3, num_vms: int = 1 << 18, num_distinct: int | None = None,
            budget: int = ROLLOUT_BUDGET, workers: int = 1) -> Batch:
    """Array-program rollouts: counted-loop programs over an input array of 1,024
    words uniform on [-2^15, 2^15), lowered to the classic RASP (about 128 to
    384 instructions each), memory 2,048 words, output capacity 1,024, budget
    2^20.  `num_distinct` program structures are generated (program v has
    structure v mod num_distinct; default: every machine its own program);
    every machine has its own input array.  Draw order: structures by
    (seed, index) streams; tapes (N x 1024) from PCG64(seed).  Structures are
    lowered in chunks of 4,096 (in `workers` spawned processes when it is
    above 1; the result does not depend on it)."""
    distinct = num_vms if num_distinct is None else min(num_distinct, num_vms)
    chunk = 4096
    jobs = [(seed, a, min(distinct, a + chunk)) for a in range(0, distinct, chunk)]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            parts = pool.map(_rollout_chunk, jobs)
    else:
        parts = [_rollout_chunk(j) for j in jobs]
    progs = [p for part in parts for p in part]
    which = np.arange(num_vms) % len(progs)
    plen = np.array([len(progs[w]) for w in which], dtype=np.int64)
    prog = np.concatenate([progs[w] for w in which])
    rng = np.random.Generator(np.random.PCG64(seed))
    tape = rng.integers(-(1 << 15), 1 << 15, size=(num_vms, ROLLOUT_ARRAY), dtype=np.int32)
    return Batch(ISA_CLASSIC, prog, _offsets(plen), np.full(num_vms, ROLLOUT_MEM, np.uint32),
                 tape.reshape(-1), np.arange(num_vms + 1, dtype=np.uint64) * np.uint64(ROLLOUT_ARRAY),
                 np.full(num_vms, ROLLOUT_ARRAY, np.uint32),
                 np.full(num_vms, ROLLOUT_OUT, np.uint32), budget=budget,
                 name="rollouts %dx[128,384] n=2048 budget=2^20" % num_vms,
                 meta=dict(seed=seed, num_distinct=len(progs)))


# ---- Sec. 3: uniform Sec. 2.2 programs of exactly L terminals (Fig. 1 workload) ----

FIG1_L = 100
FIG1_N, FIG1_ELL, FIG1_S, FIG1_MU = 250, 10, 2, 10
FIG1_BUDGET = 10 ** 6


def fig1_source(seed: int, index: int, L: int = FIG1_L) -> str:
    """Source text of program `index` of the family `seed` (independent of N):
    uniform over the Sec. 2.2 programs of exactly L terminals, drawn from
    Python's Mersenne Twister seeded with seed * 2^40 + index."""
    return grammar.sample_program(L, random.Random(seed * (1 << 40) + index))


def _fig1_chunk(job):
    seed, start, stop, L = job
    progs, arity = [], []
    for v in range(start, stop):
        pairs, lay = dsl.lower_word(dsl.parse(fig1_source(seed, v, L)), ell=FIG1_ELL, s=FIG1_S,
                                    mu=FIG1_MU, read_inputs=True)
        if 2 * len(pairs) + lay.data_words > FIG1_N:
            raise RuntimeError("program %d does not fit n = %d" % (v, FIG1_N))
        progs.append(np.array(dsl.flatten(pairs), dtype=np.int32))
        arity.append(lay.length["ipt"])
    return progs, arity


def fig1(seed: int = 5, num_vms: int = 1 << 18, L: int = FIG1_L, budget: int = FIG1_BUDGET,
         workers: int = 1) -> Batch:
    """The Sec. 3 evaluation: word-RASP machines with w = 32, n = 250, l = 10,
    s = 2, each running a program drawn uniformly from the Sec. 2.2 snippets of
    exactly L = 100 terminals (``grammar``), lowered by the Sec. 2.2 rules with
    scr of mu = 10 words and a prologue that READs the input into ipt.  The
    input x is arity(P) words uniform over all 2^32 values (x ~ F_2^(w arity)),
    from PCG64(seed) in machine order; budget tau_max = 10^6.  Programs are
    generated in chunks of 4,096 (in `workers` spawned processes when it is
    above 1, which needs a __main__ that is a file; the result does not
    depend on it)."""
    chunk = 4096
    jobs = [(seed, a, min(num_vms, a + chunk), L) for a in range(0, num_vms, chunk)]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            parts = pool.map(_fig1_chunk, jobs)
    else:
        parts = [_fig1_chunk(j) for j in jobs]
    progs = [p for part in parts for p in part[0]]
    arity = np.array([a for part in parts for a in part[1]], dtype=np.int64)
    plen = np.array([len(p) for p in progs], dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(seed))
    tape = rng.integers(-(1 << 31), 1 << 31, size=int(arity.sum()), dtype=np.int64).astype(np.int32)
    return Batch(ISA_WORD, np.concatenate(progs), _offsets(plen),
                 np.full(num_vms, FIG1_N, np.uint32), tape, _offsets(arity),
                 np.full(num_vms, FIG1_ELL, np.uint32), np.full(num_vms, FIG1_S, np.uint32),
                 budget=budget, name="fig1 %d x L=%d n=250 budget=10^6" % (num_vms, L),
                 meta=dict(seed=seed, L=L))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4}


def save_batch(b: Batch, path: str) -> None:
    """Write a batch to an .npz file (numpy arrays and a JSON header)."""
    import json
    header = json.dumps(dict(isa=int(b.isa), budget=int(b.budget), name=b.name, word_bits=int(b.word_bits),
                             meta={k: v for k, v in b.meta.items() if isinstance(v, (int, float, str))}))
    tmp = path + ".tmp.npz"
    np.savez(tmp, header=np.frombuffer(header.encode(), dtype=np.uint8), prog=b.prog, prog_off=b.prog_off,
             mem_words=b.mem_words, tape=b.tape, tape_off=b.tape_off, tape_cap=b.tape_cap, out_cap=b.out_cap)
    import os
    os.replace(tmp, path)


def load_batch(path: str) -> Batch:
    """Read a batch written by save_batch (no pickled objects)."""
    import json
    with np.load(path, allow_pickle=False) as z:
        h = json.loads(bytes(z["header"]).decode())
        return Batch(h["isa"], z["prog"], z["prog_off"], z["mem_words"], z["tape"], z["tape_off"],
                     z["tape_cap"], z["out_cap"], budget=h["budget"], name=h["name"], meta=h["meta"],
                     word_bits=h["word_bits"])
