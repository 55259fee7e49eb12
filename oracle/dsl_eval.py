"""Direct evaluation of array programs -- TEST INFRASTRUCTURE.

The plain meaning of the programs that the front end lowers to RASP: walk the
AST and update arrays, no machine involved.  A lowered program run on the RASP
must print exactly what this evaluator returns (Sec. 2.2 assigns the array
language its meaning through the lowering rules; this is the same meaning
stated directly).

Two languages, both given as plain nested tuples:

* the Sec. 2.2 array language: arrays ipt (min(declared, l) words), opt
  (min(declared, s) words) and scr (mu words), indexed modulo their length; + and * are
  word operations mod 2^w; ``ife G`` takes the first block when G is non-zero;
  ``whl G`` repeats while G is non-zero; ``hlt`` and the end of the body both
  print opt[0..l) and stop.
* the counted-loop rollout language: read the whole input array (tape word t
  into element len-1-t), then for each pass walk k = len-1 down to 0 with
  x = arr[k], run the body, and print every accumulator after the pass.
  Values are unbounded integers (the generator bounds them statically).

Output is truncated to the machine's output capacity s, the bounded append of
Sec. 2.1.
"""
from __future__ import annotations


class _Halt(Exception):
    pass


class OutOfFuel(Exception):
    pass


def eval_paper(fun, w=32, ipt=None, mu=10, s=2, ell=10, fuel=10 ** 7):
    """Evaluate a Sec. 2.2 program; returns the printed words (at most s).

    The arrays have the sizes that the typing of Sec. 2.2 allows: ipt holds
    min(declared, l) words and opt min(declared, s) words (ipt: W^(k <= l),
    opt: W^(e <= s)); ``ipt`` gives the input words (missing ones are zero)."""
    _, n_in, n_out, body = fun
    mask = (1 << w) - 1
    sign = 1 << (w - 1)

    def word(v):
        v &= mask
        return v - (1 << w) if v & sign else v

    k_in, k_out = min(n_in, ell), min(n_out, s)
    given = list(ipt or [])[:k_in]
    arrs = {"ipt": [word(v) for v in given] + [0] * (k_in - len(given)),
            "opt": [0] * k_out, "scr": [0] * mu}
    left = [fuel]

    def tick():
        left[0] -= 1
        if left[0] < 0:
            raise OutOfFuel()

    def get(arr, z):
        a = arrs[arr]
        return a[z % len(a)]

    def val(e):
        if e[0] == "get":
            return get(e[1], e[2])
        if e[0] == "const":
            return e[1]
        lhs, rhs = val(e[1]), val(e[2])
        return word(lhs + rhs) if e[0] == "add" else word(lhs * rhs)

    def run(block):
        for st in block:
            tick()
            if st[0] == "put":
                a = arrs[st[1][0]]
                a[st[1][1] % len(a)] = val(st[2])
            elif st[0] == "ife":
                run(st[2] if get(*st[1]) != 0 else st[3])
            elif st[0] == "whl":
                while get(*st[1]) != 0:
                    tick()
                    run(st[2])
            elif st[0] == "hlt":
                raise _Halt()

    try:
        run(body)
    except _Halt:
        pass
    return list(arrs["opt"])


def eval_counted(prog, tape, s):
    """Evaluate a counted-loop rollout program on its input tape."""
    _, n_acc, alen, passes, _ = prog
    arr = [0] * alen
    for t in range(alen):
        arr[alen - 1 - t] = tape[t] if t < len(tape) else 0
    acc = [0] * n_acc
    out = []

    def operand(op, x):
        if op[0] == "x":
            return x
        if op[0] == "k":
            return op[1]
        return 0

    def cond(c, x):
        if c[0] == "x":
            return x > 0
        if c[0] == "acc":
            return acc[c[1]] > 0
        return acc[c[1]] - x > 0

    def run(body, x):
        for st in body:
            if st[0] == "acc":
                _, r, src, sg, op = st
                acc[r] = acc[src] + sg * operand(op, x)
            elif st[0] == "print":
                out.append(acc[st[1]])
            else:
                run(st[2] if cond(st[1], x) else st[3], x)

    for p in passes:
        for k in range(alen - 1, -1, -1):
            run(p[1], arr[k])
        out.extend(acc)
    return out[:s]
