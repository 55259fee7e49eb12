"""The RASP over unbounded integers -- TEST INFRASTRUCTURE.

Sec. 1.1 defines the RASP over Z: i, a and memory words are integers with no
wraparound.  This interpreter keeps Python integers and never reduces them; it
raises an ``overflow`` flag as soon as a value that a 32-bit machine would have
to store (i, a, a memory word) leaves [-2^31, 2^31).  On every machine whose run
never sets the flag, the 32-bit word machine of Sec. 2.1 must produce the very
same configuration, which is how the tests show that fixed-width words
coincide with Z on the generated inputs.

Same instruction sets and readings as the C oracle (circular memory by the
Euclidean remainder, immediate LOD, RD stuck once the tape is used up, bounded
output append, JMP = 8 in the classic set), but written independently: here the
machine is stuck exactly when the Sec. 1.1 table offers no case that moves it,
i.e. an unknown opcode, a read with no unread input, or a taken jump whose
target is the current instruction.
"""
from __future__ import annotations

LO, HI = -(1 << 31), (1 << 31)

WORD, CLASSIC = 0, 1


def zrun(isa, prog, tape, n, l, s, budget, start=None):
    """Run one machine for at most `budget` transitions over Z.

    prog: list of ints (2m <= n words, stored at M[0..2m)); tape: |x| <= l ints.
    start: optional dict(i, a, M, u0, y0, Y) to resume from.
    Returns dict(i, a, M, u0, y0, Y, steps, halted, overflow).
    """
    if start is None:
        M = list(prog) + [0] * (n - len(prog))
        T = list(tape) + [0] * (l - len(tape))
        i, a, u0, y0, Y = 0, 0, 0, 0, [0] * s
    else:
        M, T = list(start["M"]), list(start["T"])
        i, a, u0, y0, Y = start["i"], start["a"], start["u0"], start["y0"], list(start["Y"])
    overflow = False

    def chk(v):
        nonlocal overflow
        if not (LO <= v < HI):
            overflow = True
        return v

    steps = 0
    halted = False
    while True:
        o = M[i % n]            # Python's % on a positive modulus is Euclidean
        j = M[(i + 1) % n]
        if isa == WORD:
            ops = {1: "LOD", 2: "ADD", 3: "MUL", 4: "STO", 5: "BNZ", 6: "RD", 7: "PRI"}
        else:
            ops = {1: "LOD", 2: "ADD", 3: "SUB", 4: "STO", 5: "BPA", 6: "RD", 7: "PRI", 8: "JMP"}
        op = ops.get(o)
        if op is None:
            halted = True
        elif op == "RD" and u0 >= l:
            halted = True
        elif op == "JMP" and j == i:
            halted = True
        elif op == "BPA" and a > 0 and j == i:
            halted = True
        elif op == "BNZ" and a != 0 and j == i:
            halted = True
        if halted or steps == budget:
            break
        if op == "LOD":
            a = chk(j); i = chk(i + 2)
        elif op == "ADD":
            a = chk(a + M[j % n]); i = chk(i + 2)
        elif op == "SUB":
            a = chk(a - M[j % n]); i = chk(i + 2)
        elif op == "MUL":
            a = chk(a * M[j % n]); i = chk(i + 2)
        elif op == "STO":
            M[j % n] = a; i = chk(i + 2)
        elif op == "BPA":
            i = j if a > 0 else chk(i + 2)
        elif op == "BNZ":
            i = j if a != 0 else chk(i + 2)
        elif op == "JMP":
            i = j
        elif op == "RD":
            M[j % n] = T[u0]; u0 += 1; i = chk(i + 2)
        elif op == "PRI":
            if y0 < s:
                Y[y0] = M[j % n]; y0 += 1
            i = chk(i + 2)
        steps += 1
    return dict(i=i, a=a, M=M, u0=u0, y0=y0, Y=Y, steps=steps,
                halted=halted, overflow=overflow)
