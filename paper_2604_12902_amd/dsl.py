"""Front end: the heapless array language of Sec. 2.2 and its lowering to RASP.

This module produces *programs* (input data for the step loop); it holds none
of the step semantics.  Two languages are lowered here:

1. The paper's array language (Sec. 2.2 grammar), lowered to the word RASP by
   the Sec. 2.2 rules: Get, Put, the + and * rules through the reserved cell
   nu, Ife, While, Seq, Halt and Fun, with JMP desugared as ``LOD 1; BNZ l`` and
   HLT as the invalid pair ``0 0``.  Used to build the App. B busy beavers.

2. A counted-loop array language of this project's own design (not in the
   paper), lowered to the classic RASP (LOD/ADD/SUB/STO/BPA/RD/PRI/JMP).  It
   generates the structured array-program rollouts: a counted loop READs the
   input array into memory through self-modified operands (the stored-program
   property of Sec. 1/2), then further counted loops walk the array with nested
   if-else on signs and update accumulators.  Every value is bounded
   statically so that it fits in 32 bits.

ASTs are plain nested tuples so that an independent evaluator can consume them.

Paper language AST
  ('fun', n_in, n_out, block)          block = tuple of statements
  ('put', (arr, z), expr)              arr in {'scr', 'opt'}
  ('ife', (arr, z), then_block, else_block)
  ('whl', (arr, z), block)
  ('hlt',)
  expr: ('get', arr, z) | ('const', z) | ('add', g, e) | ('mul', g, e)
"""
from __future__ import annotations

import re

# ---- opcode numbers (shared numbering of Sec. 1.1 and Sec. 2.1) -----------------
# word RASP (Sec. 2.1)
W_LOD, W_ADD, W_MUL, W_STO, W_BNZ, W_RD, W_PRI = 1, 2, 3, 4, 5, 6, 7
# classic RASP (Sec. 1.1, plus JMP)
C_HALT, C_LOAD, C_ADD, C_SUB, C_STORE, C_JPOS, C_READ, C_PRINT, C_JMP = 0, 1, 2, 3, 4, 5, 6, 7, 8

# ---- tokenizer / parser for the Sec. 2.2 grammar ------------------------------------

_TOK = re.compile(r"\s*(->|[A-Za-z_][A-Za-z_0-9]*|\d+|[()\[\]{}:^;=+*])")


def tokenize(src: str):
    pos, out = 0, []
    src = src.strip()
    while pos < len(src):
        m = _TOK.match(src, pos)
        if not m:
            raise SyntaxError("bad character at %r" % src[pos:pos + 10])
        out.append(m.group(1))
        pos = m.end()
        while pos < len(src) and src[pos].isspace():
            pos += 1
    return out


class _Parser:
    def __init__(self, toks):
        self.t, self.k = toks, 0

    def peek(self):
        return self.t[self.k] if self.k < len(self.t) else None

    def eat(self, want=None):
        tok = self.peek()
        if tok is None or (want is not None and tok != want):
            raise SyntaxError("expected %r, got %r" % (want, tok))
        self.k += 1
        return tok

    def num(self):
        tok = self.eat()
        if not tok.isdigit():
            raise SyntaxError("expected a digit, got %r" % tok)
        return int(tok)

    def fun(self):
        self.eat("fun"); self.eat("f0"); self.eat("(")
        self.eat("ipt"); self.eat(":"); self.eat("W"); self.eat("^")
        n_in = self.num()
        self.eat(")"); self.eat("->"); self.eat("W"); self.eat("^")
        n_out = self.num()
        self.eat("{")
        body = self.block()
        self.eat("}")
        if self.peek() is not None:
            raise SyntaxError("trailing tokens")
        return ("fun", n_in, n_out, body)

    def block(self):
        if self.peek() == "hlt":
            self.eat()
            return (("hlt",),)
        stmts = [self.stmt()]
        while self.peek() == ";":
            self.eat(";")
            if self.peek() == "hlt":
                self.eat()
                stmts.append(("hlt",))
                break
            stmts.append(self.stmt())
        return tuple(stmts)

    def ref(self):
        arr = self.eat()
        if arr not in ("ipt", "scr", "opt"):
            raise SyntaxError("expected an array, got %r" % arr)
        self.eat("[")
        z = self.num()
        self.eat("]")
        return (arr, z)

    def stmt(self):
        tok = self.peek()
        if tok == "ife":
            self.eat()
            g = self.ref()
            self.eat("{"); b1 = self.block(); self.eat("}")
            self.eat("{"); b2 = self.block(); self.eat("}")
            return ("ife", g, b1, b2)
        if tok == "whl":
            self.eat()
            g = self.ref()
            self.eat("{"); b = self.block(); self.eat("}")
            return ("whl", g, b)
        dst = self.ref()
        if dst[0] == "ipt":
            raise SyntaxError("ipt is not assignable")
        self.eat("=")
        return ("put", dst, self.expr())

    def expr(self):
        if self.peek().isdigit():
            return ("const", self.num())
        g = ("get",) + self.ref()
        if self.peek() in ("+", "*"):
            op = "add" if self.eat() == "+" else "mul"
            rhs = ("const", self.num()) if self.peek().isdigit() else ("get",) + self.ref()
            return (op, g, rhs)
        return g


def parse(src: str):
    """Parse one ``fun f0 (...) -> ... { ... }`` program of the Sec. 2.2 grammar."""
    return _Parser(tokenize(src)).fun()


# ---- Sec. 2.2 lowering to the word RASP ----------------------------------------------

class Layout:
    """Data regions placed after the program (Sec. 2.2).

    Cell 2m + 0 is the reserved nu; cells 2m+1..2m+4 are left reserved (the
    paper budgets 5 reserved words); then ipt (l words), opt (s words) and scr
    (mu words).  Array indexing is modulo the array's length.  Sec. 2.2 types
    the arrays as ipt : W^(k <= l) and opt : W^(e <= s); a program that declares
    more (the grammar allows arities up to 9) gets the region's size, so the
    regions stay disjoint: |ipt| = min(declared, l), |opt| = min(declared, s)."""

    def __init__(self, n_in, n_out, ell, s, mu):
        if ell < 1 or s < 1 or mu < 1:
            raise ValueError("the ipt, opt and scr regions need at least one word each")
        self.n_in, self.n_out, self.ell, self.s, self.mu = n_in, n_out, ell, s, mu
        self.base = {"ipt": 5, "opt": 5 + ell, "scr": 5 + ell + s}
        self.length = {"ipt": min(n_in, ell), "opt": min(n_out, s), "scr": mu}

    def offset(self, arr, z):
        return self.base[arr] + (z % self.length[arr])

    @property
    def data_words(self):
        return 5 + self.ell + self.s + self.mu


def lower_word(fun, ell=10, s=2, mu=10, read_inputs=False):
    """Lower a parsed program to word-RASP (opcode, operand) pairs.

    Returns (pairs, layout).  Operands are resolved to absolute word addresses
    (instruction k sits at words 2k, 2k+1; a jump target is a word address).
    With read_inputs, a prologue ``RD ipt[k]`` for k < |ipt| moves the input
    word x_k from the tape (where c0 of Sec. 2.1 puts x) into the ipt region;
    without it ipt stays zero, as in the App. B search."""
    _, n_in, n_out, body = fun
    lay = Layout(n_in, n_out, ell, s, mu)
    code = []           # items: (op, operand) with operand int | ('d', off) | ('L', id)
    labels = {}
    counter = [0]

    def new_label():
        counter[0] += 1
        return counter[0]

    def mark(lbl):
        labels[lbl] = len(code)

    def emit(op, arg):
        code.append((op, arg))

    def jmp(lbl):                       # JMP l  ==  LOD 1; BNZ l
        emit(W_LOD, 1); emit(W_BNZ, ("L", lbl))

    def hlt():                          # PRI q_i for every output, then HLT = 0 0
        for q in range(lay.length["opt"]):
            emit(W_PRI, ("d", lay.offset("opt", q)))
        emit(0, 0)

    def get(arr, z):                    # Get: LOD 0; ADD [alpha]_z
        emit(W_LOD, 0); emit(W_ADD, ("d", lay.offset(arr, z)))

    def value(e):                       # E =>_a A
        kind = e[0]
        if kind == "get":
            get(e[1], e[2])
        elif kind == "const":
            emit(W_LOD, e[1])
        else:                           # J1 STO nu J2 (ADD|MUL) nu
            value(e[1])
            emit(W_STO, ("d", 0))
            value(e[2])
            emit(W_ADD if kind == "add" else W_MUL, ("d", 0))

    def block(b):
        for st in b:
            stmt(st)

    def stmt(st):
        kind = st[0]
        if kind == "put":
            value(st[2])
            emit(W_STO, ("d", lay.offset(*st[1])))
        elif kind == "ife":             # J BNZ lt C2 JMP le lt: C1 le:
            lt, le = new_label(), new_label()
            get(*st[1]); emit(W_BNZ, ("L", lt))
            block(st[3]); jmp(le)
            mark(lt); block(st[2]); mark(le)
        elif kind == "whl":             # lh: J BNZ lb JMP le lb: C JMP lh le:
            lh, lb, le = new_label(), new_label(), new_label()
            mark(lh); get(*st[1]); emit(W_BNZ, ("L", lb)); jmp(le)
            mark(lb); block(st[2]); jmp(lh); mark(le)
        elif kind == "hlt":
            hlt()
        else:
            raise ValueError(kind)

    if read_inputs:
        for k in range(lay.length["ipt"]):
            emit(W_RD, ("d", lay.offset("ipt", k)))
    block(body)
    hlt()                               # Fun: C PRI q_0..q_{l-1} HLT
    m = len(code)
    pairs = []
    for op, arg in code:
        if isinstance(arg, tuple) and arg[0] == "d":
            arg = 2 * m + arg[1]
        elif isinstance(arg, tuple) and arg[0] == "L":
            arg = 2 * labels[arg[1]]
        pairs.append((op, arg))
    return pairs, lay


def flatten(pairs):
    out = []
    for op, arg in pairs:
        out.extend((int(op), int(arg)))
    return out


# ---- counted-loop array language, lowered to the classic RASP ------------------------
#
# AST (this project's own language for the rollout workload):
#   ('prog', n_acc, array_len, passes, prints_per_pass)
#   pass  = ('pass', body)              a counted loop over the array, k = len-1 .. 0
#   body  = tuple of statements, each:
#     ('acc', r, src, sign, operand)    acc_r = acc_src + sign * operand
#                                       operand: ('x',) the current element,
#                                                ('k', c) a constant, ('z',) zero
#     ('if', cond, then_body, else_body) cond: ('x',)  x > 0
#                                              ('acc', r)  acc_r > 0
#                                              ('diff', r) acc_r - x > 0
#     ('print', r)                      append acc_r to the output
# The program first reads the whole input array, element k from tape word
# len-1-k (a counted loop of READs whose target operand is patched each
# iteration), then runs its passes, printing every accumulator after each pass,
# and halts.

class ClassicLayout:
    def __init__(self, prog_words, n_acc, array_len):
        base = prog_words
        self.one = base                  # constant 1
        self.ctr = base + 1              # loop counter
        self.nu = base + 2               # temporary
        self.x = base + 3                # current element
        self.acc0 = base + 4             # accumulators
        self.arr = base + 4 + n_acc      # array region
        self.end = self.arr + array_len


def lower_classic(prog):
    """Lower a counted-loop program to classic-RASP (opcode, operand) pairs.

    Returns (pairs, data_words_after_program)."""
    _, n_acc, alen, passes, _ = prog
    code, labels, counter = [], {}, [0]

    def new_label():
        counter[0] += 1
        return counter[0]

    def mark(l):
        labels[l] = len(code)

    def emit(op, arg):
        code.append((op, arg))

    # symbolic data cells, resolved once the program length is known
    ONE, CTR, NU, X = ("c", "one"), ("c", "ctr"), ("c", "nu"), ("c", "x")

    def ACC(r):
        return ("acc", r)

    def ARRM1():                         # address of arr[-1]
        return ("arr", -1)

    def counted_loop(body_fn):
        # ctr = alen; while ctr > 0 { body; ctr = ctr - 1 }
        lh, lb, le = new_label(), new_label(), new_label()
        emit(C_LOAD, alen); emit(C_STORE, CTR)
        mark(lh)
        emit(C_LOAD, 0); emit(C_ADD, CTR); emit(C_JPOS, ("L", lb)); emit(C_JMP, ("L", le))
        mark(lb)
        body_fn()
        emit(C_LOAD, 0); emit(C_ADD, CTR); emit(C_SUB, ONE); emit(C_STORE, CTR)
        emit(C_JMP, ("L", lh))
        mark(le)

    def patch_operand(target):
        # operand word of instruction `target` <- address of arr[ctr - 1]
        emit(C_LOAD, ARRM1()); emit(C_ADD, CTR)
        emit(C_STORE, ("self", target))

    def load_body():
        patch_operand(len(code) + 3)     # the READ right after the patch
        emit(C_READ, 0)                  # operand patched to arr[ctr-1]

    def fetch_x():
        patch_operand(len(code) + 4)     # the ADD after the patch and LOAD 0
        emit(C_LOAD, 0)
        emit(C_ADD, 0)                   # operand patched to arr[ctr-1]
        emit(C_STORE, X)

    def value_into_a(src, sign, operand):
        # a = acc_src + sign * operand
        if operand[0] == "z":
            emit(C_LOAD, 0); emit(C_ADD, ACC(src))
            return
        if operand[0] == "x":
            emit(C_LOAD, 0); emit(C_ADD, ACC(src))
            emit(C_ADD if sign > 0 else C_SUB, X)
            return
        # constant: a = acc_src + sign*c   via   LOAD c; STO nu; LOAD 0; ADD acc; ADD/SUB nu
        emit(C_LOAD, operand[1]); emit(C_STORE, NU)
        emit(C_LOAD, 0); emit(C_ADD, ACC(src))
        emit(C_ADD if sign > 0 else C_SUB, NU)

    def cond_into_a(cond):
        if cond[0] == "x":
            emit(C_LOAD, 0); emit(C_ADD, X)
        elif cond[0] == "acc":
            emit(C_LOAD, 0); emit(C_ADD, ACC(cond[1]))
        else:                            # acc_r - x
            emit(C_LOAD, 0); emit(C_ADD, ACC(cond[1])); emit(C_SUB, X)

    def body(stmts):
        for st in stmts:
            if st[0] == "acc":
                _, r, src, sign, operand = st
                value_into_a(src, sign, operand)
                emit(C_STORE, ACC(r))
            elif st[0] == "print":
                emit(C_PRINT, ACC(st[1]))
            elif st[0] == "if":          # cond JPOS lt  else-part JMP le  lt: then-part  le:
                lt, le = new_label(), new_label()
                cond_into_a(st[1]); emit(C_JPOS, ("L", lt))
                body(st[3]); emit(C_JMP, ("L", le))
                mark(lt); body(st[2]); mark(le)
            else:
                raise ValueError(st[0])

    # prologue: one = 1
    emit(C_LOAD, 1); emit(C_STORE, ONE)
    counted_loop(load_body)
    for p in passes:
        counted_loop(lambda p=p: (fetch_x(), body(p[1])))
        for r in range(n_acc):
            emit(C_PRINT, ACC(r))
    emit(C_HALT, 0)

    m = len(code)
    lay = ClassicLayout(2 * m, n_acc, alen)
    named = {"one": lay.one, "ctr": lay.ctr, "nu": lay.nu, "x": lay.x}
    pairs = []
    for op, arg in code:
        if isinstance(arg, tuple):
            kind = arg[0]
            if kind == "c":
                arg = named[arg[1]]
            elif kind == "acc":
                arg = lay.acc0 + arg[1]
            elif kind == "arr":
                arg = lay.arr + arg[1]
            elif kind == "L":
                arg = 2 * labels[arg[1]]
            elif kind == "self":
                arg = 2 * arg[1] + 1     # the operand word of instruction arg[1]
            else:
                raise ValueError(kind)
        pairs.append((op, arg))
    return pairs, lay.end - 2 * m
