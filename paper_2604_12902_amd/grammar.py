"""Uniform sampler of Sec. 2.2 array programs with exactly L terminals.

Sec. 3 evaluates programs drawn uniformly from the valid snippets of the Sec. 2.2
grammar of one fixed length.  This module counts, for every nonterminal and
every length k, the derivations that yield exactly k terminals (the terminals
are the whitespace-separated symbols of the grammar, "->" being one), and then
samples a derivation top-down, choosing each production with probability
proportional to the number of completions it leaves.  Counts are exact Python
integers and every choice is an exact integer draw (``randrange``), so each
program of length L is equally likely.  The grammar is unambiguous (B is
right-recursive; an expression is fixed by its first two terminals), so
uniform over derivations is uniform over strings.

Input generation only: nothing here runs a machine.
"""
from __future__ import annotations

import random
from functools import lru_cache

DIGITS_N = tuple(str(d) for d in range(1, 10))      # N ::= 1 | ... | 9
DIGITS_Z = ("0",) + DIGITS_N                         # Z ::= 0 | N
READ_ARRAYS = ("ipt", "scr", "opt")                  # G
WRITE_ARRAYS = ("scr", "opt")                        # P
FUN_TERMINALS = 15       # fun f0 ( ipt : W ^ N ) -> W ^ N { ... }

# E ::= G + G | G * G | G + Z | G * Z | G | Z  ->  {length: count}
_E = {9: 2 * 30 * 30, 6: 2 * 30 * 10, 4: 30, 1: 10}


@lru_cache(maxsize=None)
def count_B(k: int) -> int:
    """Derivations of B ::= S | S ; B | hlt with exactly k terminals."""
    if k <= 0:
        return 0
    c = count_S(k) + (1 if k == 1 else 0)
    for a in range(1, k - 1):                      # S (a terminals) ; B (k - a - 1)
        c += count_S(a) * count_B(k - a - 1)
    return c


@lru_cache(maxsize=None)
def count_S(k: int) -> int:
    """Derivations of S ::= P = E | ife G { B } { B } | whl G { B }."""
    if k <= 0:
        return 0
    c = 20 * _E.get(k - 5, 0)                       # P (4) = (1) E
    c += 30 * count_B(k - 7)                         # whl G (5) { B } (2)
    for b1 in range(1, k - 9):                       # ife G (5) {B} {B} (4)
        c += 30 * count_B(b1) * count_B(k - 9 - b1)
    return c


def count_F(L: int) -> int:
    """Programs ``fun f0 ( ipt : W ^ N ) -> W ^ N { B }`` with exactly L terminals."""
    return 81 * count_B(L - FUN_TERMINALS)


class _Sampler:
    def __init__(self, rng: random.Random):
        self.rng = rng

    def pick(self, seq):
        return seq[self.rng.randrange(len(seq))]

    def G(self, out):
        out += [self.pick(READ_ARRAYS), "[", self.pick(DIGITS_Z), "]"]

    def E(self, m, out):
        r = self.rng.randrange(_E[m])
        if m == 1:
            out.append(DIGITS_Z[r])
        elif m == 4:
            self.G(out)
        elif m == 6:
            self.G(out)
            out += ["+" if r < 300 else "*", self.pick(DIGITS_Z)]
        else:
            self.G(out)
            out.append("+" if r < 900 else "*")
            self.G(out)

    def S(self, k, out):
        r = self.rng.randrange(count_S(k))
        c = 20 * _E.get(k - 5, 0)
        if r < c:
            out += [self.pick(WRITE_ARRAYS), "[", self.pick(DIGITS_Z), "]", "="]
            self.E(k - 5, out)
            return
        r -= c
        c = 30 * count_B(k - 7)
        if r < c:
            out.append("whl")
            self.G(out)
            out.append("{")
            self.B(k - 7, out)
            out.append("}")
            return
        r -= c
        for b1 in range(1, k - 9):
            c = 30 * count_B(b1) * count_B(k - 9 - b1)
            if r < c:
                out.append("ife")
                self.G(out)
                out.append("{")
                self.B(b1, out)
                out += ["}", "{"]
                self.B(k - 9 - b1, out)
                out.append("}")
                return
            r -= c
        raise AssertionError("count_S out of step with the sampler")

    def B(self, k, out):
        r = self.rng.randrange(count_B(k))
        c = count_S(k)
        if r < c:
            self.S(k, out)
            return
        r -= c
        if k == 1:
            if r == 0:
                out.append("hlt")
                return
            r -= 1
        for a in range(1, k - 1):
            c = count_S(a) * count_B(k - a - 1)
            if r < c:
                self.S(a, out)
                out.append(";")
                self.B(k - a - 1, out)
                return
            r -= c
        raise AssertionError("count_B out of step with the sampler")


def sample_program(L: int, rng: random.Random) -> str:
    """One program of exactly L terminals, uniform over the grammar's strings."""
    if count_F(L) == 0:
        raise ValueError("no program has exactly %d terminals" % L)
    s = _Sampler(rng)
    out = ["fun", "f0", "(", "ipt", ":", "W", "^", s.pick(DIGITS_N), ")", "->", "W", "^",
           s.pick(DIGITS_N), "{"]
    s.B(L - FUN_TERMINALS, out)
    out.append("}")
    return " ".join(out)
