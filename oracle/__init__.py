"""Plain CPU oracle for the RASP step loop -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never imports
it; the two meet only in the seeded input generators, which hold none of the
step semantics.

Contents
  * ``rasp_oracle.c`` (built here with gcc into ``_build/liboracle.so``): the
    serial interpreter.  Per machine it computes Phi^B(c0(P, x)) of Sec. 2, the
    number of transitions retired (the halting number tau_h of Sec. 3, capped at
    B) and whether the final configuration is a fixed point (F, Sec. 1.1/2.1).
  * ``zinterp``: the same machine over unbounded integers (Sec. 1.1 works over
    Z), used to show that 32-bit words coincide with Z on the generated inputs.
  * ``dsl_eval``: a direct evaluator of the heapless array language of
    Sec. 2.2, the plain meaning that compiled programs must reproduce.

Batches are duck-typed: any object with the attributes ``isa, prog, prog_off,
mem_words, tape, tape_off, tape_cap, out_cap`` (numpy arrays as produced by the
workload generators) is accepted.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rasp_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")

ISA_WORD = 0
ISA_CLASSIC = 1
RUNNING = 0
HALTED = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, plain C, pthreads)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    u64 = ctypes.c_uint64
    lib.or_step_full.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint32, P, P]
    lib.or_step_full.restype = None
    lib.or_c0.argtypes = [ctypes.c_int, u64] + [P] * 19
    lib.or_c0.restype = ctypes.c_int
    lib.or_advance.argtypes = [ctypes.c_int, ctypes.c_int, u64, u64, ctypes.c_int] + [P] * 15
    lib.or_advance.restype = ctypes.c_int
    lib.or_advance_mix.argtypes = [ctypes.c_int, ctypes.c_int, u64, u64, ctypes.c_int] + [P] * 16
    lib.or_advance_mix.restype = ctypes.c_int
    lib.or_fnv1a64.argtypes = [P, u64]
    lib.or_fnv1a64.restype = u64
    lib.or_digest_batch.argtypes = [u64, P, P, P, P]
    lib.or_digest_batch.restype = None
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes.astype(np.uint64), out=off[1:])
    return off


@dataclass
class State:
    """Configurations of N machines, struct-of-arrays, host memory."""
    isa: int
    w: int
    i: np.ndarray          # int32[N]
    a: np.ndarray          # int32[N]
    u0: np.ndarray         # uint32[N]
    y0: np.ndarray         # uint32[N]
    steps: np.ndarray      # uint64[N]
    status: np.ndarray     # uint8[N]
    mem: np.ndarray        # int32[sum n]
    mem_off: np.ndarray    # uint64[N+1]
    n: np.ndarray          # uint32[N]
    tape: np.ndarray       # int32[sum l]
    t_off: np.ndarray      # uint64[N+1]
    l: np.ndarray          # uint32[N]
    Y: np.ndarray          # int32[sum s]
    y_off: np.ndarray      # uint64[N+1]
    s: np.ndarray          # uint32[N]

    @property
    def N(self) -> int:
        return len(self.i)

    def mem_of(self, v: int) -> np.ndarray:
        return self.mem[int(self.mem_off[v]):int(self.mem_off[v + 1])]

    def out_of(self, v: int) -> np.ndarray:
        return self.Y[int(self.y_off[v]):int(self.y_off[v + 1])]

    def copy(self) -> "State":
        kw = {k: (v.copy() if isinstance(v, np.ndarray) else v)
              for k, v in self.__dict__.items()}
        return State(**kw)


def _shape_arrays(batch):
    N = int(len(batch.prog_off) - 1)
    n = np.asarray(batch.mem_words, dtype=np.uint32)
    tape_off = np.asarray(batch.tape_off, dtype=np.uint64)
    tlen = (tape_off[1:] - tape_off[:-1]).astype(np.uint32)
    l = tlen if batch.tape_cap is None else np.asarray(batch.tape_cap, dtype=np.uint32)
    s = np.asarray(batch.out_cap, dtype=np.uint32)
    if n.shape == ():
        n = np.full(N, n, dtype=np.uint32)
    if l.shape == ():
        l = np.full(N, l, dtype=np.uint32)
    if s.shape == ():
        s = np.full(N, s, dtype=np.uint32)
    return N, n, l, s


def init(batch, w: int = 32) -> State:
    """c0(P, x) for every machine of the batch (Sec. 2.1)."""
    lib = _load()
    N, n, l, s = _shape_arrays(batch)
    mem_off, t_off, y_off = _offsets(n), _offsets(l), _offsets(s)
    st = State(isa=int(batch.isa), w=w,
               i=np.zeros(N, np.int32), a=np.zeros(N, np.int32),
               u0=np.zeros(N, np.uint32), y0=np.zeros(N, np.uint32),
               steps=np.zeros(N, np.uint64), status=np.zeros(N, np.uint8),
               mem=np.zeros(int(mem_off[-1]), np.int32), mem_off=mem_off, n=n,
               tape=np.zeros(int(t_off[-1]), np.int32), t_off=t_off, l=l,
               Y=np.zeros(int(y_off[-1]), np.int32), y_off=y_off, s=s)
    prog = np.ascontiguousarray(batch.prog, dtype=np.int32)
    prog_off = np.ascontiguousarray(batch.prog_off, dtype=np.uint64)
    tape = np.ascontiguousarray(batch.tape, dtype=np.int32)
    tape_off = np.ascontiguousarray(batch.tape_off, dtype=np.uint64)
    rc = lib.or_c0(w, N, _p(prog), _p(prog_off), _p(tape), _p(tape_off),
                   _p(n), _p(l), _p(s), _p(mem_off), _p(t_off), _p(y_off),
                   _p(st.i), _p(st.a), _p(st.u0), _p(st.y0), _p(st.steps), _p(st.status),
                   _p(st.mem), _p(st.tape), _p(st.Y))
    if rc != 0:
        raise ValueError("oracle: a program is longer than its memory or a tape longer than l")
    return st


def advance(st: State, budget: int, threads: int = 1) -> None:
    """Advance every machine by at most `budget` more transitions, in place."""
    lib = _load()
    rc = lib.or_advance(st.isa, st.w, st.N, int(budget), int(threads),
                        _p(st.i), _p(st.a), _p(st.u0), _p(st.y0), _p(st.steps), _p(st.status),
                        _p(st.mem), _p(st.mem_off), _p(st.n),
                        _p(st.tape), _p(st.t_off), _p(st.l),
                        _p(st.Y), _p(st.y_off), _p(st.s))
    if rc != 0:
        raise ValueError("oracle: bad arguments to or_advance")


MIX_NAMES = {1: "LOAD", 2: "ADD", 3: "SUB/MUL", 4: "STORE", 5: "JPOS/BNZ", 6: "READ",
             7: "PRINT", 8: "JMP", 9: "PRINT appended"}


def advance_mix(st: State, budget: int, threads: int = 1) -> np.ndarray:
    """advance() that also returns the retired-opcode histogram (uint64[16]):
    entry k (1..8) counts retired transitions with opcode k, entry 9 the PRINTs
    that appended an output word."""
    lib = _load()
    mix = np.zeros(16, np.uint64)
    rc = lib.or_advance_mix(st.isa, st.w, st.N, int(budget), int(threads),
                            _p(st.i), _p(st.a), _p(st.u0), _p(st.y0), _p(st.steps), _p(st.status),
                            _p(st.mem), _p(st.mem_off), _p(st.n),
                            _p(st.tape), _p(st.t_off), _p(st.l),
                            _p(st.Y), _p(st.y_off), _p(st.s), _p(mix))
    if rc != 0:
        raise ValueError("oracle: bad arguments to or_advance_mix")
    return mix


def run(batch, budget: int, w: int = 32, threads: int = 1) -> State:
    """Phi^budget(c0(P, x)) for every machine, with steps and halting status."""
    st = init(batch, w=w)
    advance(st, budget, threads=threads)
    return st


def subset(st: State, idx) -> State:
    """The machines `idx` of a state, as a state of their own (same order)."""
    idx = np.asarray(idx, dtype=np.int64)

    def gather(arr, off):
        parts = [arr[int(off[v]):int(off[v + 1])] for v in idx]
        return np.concatenate(parts) if parts else arr[:0].copy()
    n, l, s = st.n[idx], st.l[idx], st.s[idx]
    return State(isa=st.isa, w=st.w, i=st.i[idx].copy(), a=st.a[idx].copy(),
                 u0=st.u0[idx].copy(), y0=st.y0[idx].copy(),
                 steps=st.steps[idx].copy(), status=st.status[idx].copy(),
                 mem=gather(st.mem, st.mem_off), mem_off=_offsets(n), n=n,
                 tape=gather(st.tape, st.t_off), t_off=_offsets(l), l=l,
                 Y=gather(st.Y, st.y_off), y_off=_offsets(s), s=s)


def digest(st: State) -> np.ndarray:
    """FNV-1a-64 of each machine's memory words (little-endian bytes)."""
    lib = _load()
    out = np.zeros(st.N, np.uint64)
    lib.or_digest_batch(st.N, _p(st.mem), _p(st.mem_off), _p(st.n), _p(out))
    return out


def fnv1a64(words: np.ndarray) -> int:
    lib = _load()
    words = np.ascontiguousarray(words, dtype=np.int32)
    return int(lib.or_fnv1a64(_p(words), len(words)))


def step_full(isa: int, w: int, n: int, l: int, s: int, c: np.ndarray) -> np.ndarray:
    """Phi_w on one whole configuration vector [i, a, M, u0, tape, y0, Y]."""
    lib = _load()
    c = np.ascontiguousarray(c, dtype=np.int64)
    assert len(c) == n + l + s + 4
    d = np.empty_like(c)
    lib.or_step_full(isa, w, n, l, s, _p(c), _p(d))
    return d


def run_literal(isa: int, w: int, n: int, l: int, s: int, c: np.ndarray, budget: int):
    """Phi^budget by whole-vector steps; a fixed point is c == Phi_w(c).

    Returns (final vector, transitions applied, halted flag).  Slow: for tiny
    machines only, as the definitional check of the interpreter."""
    c = np.ascontiguousarray(c, dtype=np.int64)
    t = 0
    while True:
        d = step_full(isa, w, n, l, s, c)
        if np.array_equal(d, c):
            return c, t, True
        if t == budget:
            return c, t, False
        c = d
        t += 1


def vector_of(st: State, v: int) -> np.ndarray:
    """Machine v of a state as the flat configuration vector of Sec. 2.1."""
    return np.concatenate([
        np.array([st.i[v], st.a[v]], np.int64),
        st.mem_of(v).astype(np.int64),
        np.array([st.u0[v]], np.int64),
        st.tape[int(st.t_off[v]):int(st.t_off[v + 1])].astype(np.int64),
        np.array([st.y0[v]], np.int64),
        st.out_of(v).astype(np.int64)])
