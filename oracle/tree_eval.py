"""Second, independent evaluator: postfix -> expression tree -> recursion.

TEST INFRASTRUCTURE ONLY.  Written separately from ``gp_oracle.c`` (different
algorithm, different language, different overflow test) so that the two can
pin each other on brute-force sets.  Same semantics (RPN stack machine and
op table of the paper's GCL section; protected DIV/LOG/SQRT readings; fp32
overflow range emulated), fp64 arithmetic via Python's ``math``.
"""
from __future__ import annotations

import math
import struct

import numpy as np

LOAD, CONST, ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, ABS = range(12)
UNARY = {SIN, COS, EXP, LOG, SQRT, ABS}
BINARY = {ADD, SUB, MUL, DIV}
THETA = struct.unpack("f", struct.pack("f", 0.001))[0]


class Invalid(Exception):
    pass


def parse(prog, consts, n_vars, max_depth=32):
    """Build a tree (nested tuples) from a postfix node array.  Raises
    ``Invalid`` for anything that is not a valid program."""
    work = []
    for w in prog:
        w = int(w)
        op, arg = w & 0xFF, w >> 8
        if op == LOAD:
            if arg >= n_vars:
                raise Invalid("var")
            work.append(("x", arg))
        elif op == CONST:
            if arg >= len(consts):
                raise Invalid("const")
            work.append(("c", float(consts[arg])))
        elif op in UNARY:
            if not work:
                raise Invalid("underflow")
            work.append(("u", op, work.pop()))
        elif op in BINARY:
            if len(work) < 2:
                raise Invalid("underflow")
            right = work.pop()
            left = work.pop()
            work.append(("b", op, left, right))
        else:
            raise Invalid("op")
        if len(work) > max_depth:
            raise Invalid("depth")
    if len(work) != 1:
        raise Invalid("final")
    return work[0]


def _range(v):
    """fp32 overflow emulation: round-trip through an IEEE binary32 pack; a
    finite value whose fp32 rounding is infinite becomes +-inf."""
    if math.isnan(v) or math.isinf(v):
        return v
    try:
        r = struct.unpack("f", struct.pack("f", v))[0]
    except OverflowError:            # older CPython refuses instead
        r = math.inf
    if math.isinf(r):
        return math.copysign(math.inf, v)
    return v


def _sin(a):
    return math.nan if (math.isinf(a) or math.isnan(a)) else math.sin(a)


def _cos(a):
    return math.nan if (math.isinf(a) or math.isnan(a)) else math.cos(a)


def _exp(a):
    if math.isnan(a):
        return a
    try:
        return math.exp(a)
    except OverflowError:
        return math.inf


def _log(a):
    if math.isnan(a):
        return a
    m = abs(a)
    if m <= THETA:
        return 0.0
    return math.log(m)


def _div(a, b):
    # abs(nan) <= THETA is False, so a NaN divisor gives a / nan = nan
    if abs(b) <= THETA:
        return 1.0
    return a / b


def evaluate(tree, xs):
    """Value of ``tree`` for one case (``xs`` = the case's inputs)."""
    kind = tree[0]
    if kind == "x":
        return float(xs[tree[1]])
    if kind == "c":
        return tree[1]
    if kind == "u":
        a = evaluate(tree[2], xs)
        op = tree[1]
        if op == SIN:
            v = _sin(a)
        elif op == COS:
            v = _cos(a)
        elif op == EXP:
            v = _exp(a)
        elif op == LOG:
            v = _log(a)
        elif op == SQRT:
            v = math.sqrt(abs(a))
        else:
            v = abs(a)
        return _range(v)
    a = evaluate(tree[2], xs)
    b = evaluate(tree[3], xs)
    op = tree[1]
    # Python float +, -, * follow IEEE 754 (inf - inf = nan, inf * 0 = nan)
    if op == ADD:
        v = a + b
    elif op == SUB:
        v = a - b
    elif op == MUL:
        v = a * b
    else:
        v = _div(a, b)
    return _range(v)


def outputs(prog, consts, X, n_vars=None):
    """Per-case values of one program over X (variable major)."""
    X = np.asarray(X, dtype=np.float32)
    n_vars = X.shape[0] if n_vars is None else n_vars
    tree = parse(prog, consts, n_vars)
    cols = X.astype(np.float64).T
    return np.array([evaluate(tree, xs) for xs in cols], dtype=np.float64)


def to_infix(tree, names=("x0", "x1", "x2", "x3", "x4", "x5", "x6", "x7", "x8", "x9")):
    """Readable infix form (debug aid)."""
    kind = tree[0]
    if kind == "x":
        return names[tree[1]] if tree[1] < len(names) else "x%d" % tree[1]
    if kind == "c":
        return repr(tree[1])
    if kind == "u":
        nm = {SIN: "sin", COS: "cos", EXP: "exp", LOG: "plog", SQRT: "psqrt", ABS: "abs"}[tree[1]]
        return "%s(%s)" % (nm, to_infix(tree[2], names))
    sym = {ADD: "+", SUB: "-", MUL: "*", DIV: "%"}[tree[1]]
    return "(%s %s %s)" % (to_infix(tree[2], names), sym, to_infix(tree[3], names))
