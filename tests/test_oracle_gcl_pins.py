"""Pins of the oracle's full GCL command table (the paper's Table of GCL
commands): stack moves and variables against the tree programs they stand
for, the math commands against closed forms and identities, and the
validity rules against a brute-force enumeration of short programs."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import (ABS, ACOS, ADD, ASIN, ATAN, CBRT, CONST, COPY, COS, CUBE, DEL, DIV, DUP,
                    EXP, LOAD, LOG, MUL, PASTE, POW, SIGN, SIN, SQRT, SQRT_RAW, SQUARE, SUB,
                    SWAP, TAN, TANH, gcl)

MASK = oracle.MASK_GCL


def _out(prog, X, consts=None, mode=oracle.M64):
    consts = np.zeros(1, np.float32) if consts is None else np.asarray(consts, np.float32)
    return oracle.program_outputs(np.array(prog, np.uint32), consts, X, allowed_mask=MASK,
                                  mode=mode)


def _X(n=257, lo=-3.0, hi=3.0, seed=1, k=3):
    return np.random.default_rng(seed).uniform(lo, hi, (k, n)).astype(np.float32)


def L(i):
    return LOAD | (i << 8)


def C(i):
    return CONST | (i << 8)


def V(op, k):
    return op | (k << 8)


class TestStackMoves:
    """DUP, SWAP, DEL, COPY/PASTE give bit for bit the values of the tree
    programs they abbreviate (all modes)."""

    @pytest.mark.parametrize("mode", [oracle.M64, oracle.M32E])
    def test_dup(self, mode):
        X = _X()
        for op in (ADD, SUB, MUL, DIV):
            assert np.array_equal(_out([L(0), DUP, op], X, mode=mode),
                                  _out([L(0), L(0), op], X, mode=mode), equal_nan=True)
        # DUP of an inner result: (x0 + x1)^2
        assert np.array_equal(_out([L(0), L(1), ADD, DUP, MUL], X, mode=mode),
                              _out([L(0), L(1), ADD, L(0), L(1), ADD, MUL], X, mode=mode))

    @pytest.mark.parametrize("mode", [oracle.M64, oracle.M32E])
    def test_swap(self, mode):
        X = _X()
        for op in (SUB, DIV, POW):
            assert np.array_equal(_out([L(0), L(1), SWAP, op], X, mode=mode),
                                  _out([L(1), L(0), op], X, mode=mode), equal_nan=True)
        # SWAP below an untouched element
        assert np.array_equal(_out([L(2), L(0), L(1), SWAP, SUB, MUL], X, mode=mode),
                              _out([L(2), L(1), L(0), SUB, MUL], X, mode=mode))

    def test_del(self):
        X = _X()
        assert np.array_equal(_out([L(0), L(1), DEL], X), X[0].astype(np.float64))
        assert np.array_equal(_out([L(0), L(1), SIN, DEL, L(2), ADD], X),
                              _out([L(0), L(2), ADD], X))
        # the stack may run empty in between
        assert np.array_equal(_out([L(0), DEL, L(1)], X), X[1].astype(np.float64))

    @pytest.mark.parametrize("mode", [oracle.M64, oracle.M32E])
    def test_copy_paste(self, mode):
        X = _X()
        prog = [L(0), V(COPY, 3), L(1), ADD, V(PASTE, 3), MUL]
        tree = [L(0), L(1), ADD, L(0), MUL]
        assert np.array_equal(_out(prog, X, mode=mode), _out(tree, X, mode=mode))
        # nested and crossed lifetimes, a variable name used twice in turn
        prog = [L(0), V(COPY, 0), L(1), V(COPY, 5), MUL, V(PASTE, 0), SUB, V(PASTE, 5), DIV,
                L(2), V(COPY, 0), SIN, V(PASTE, 0), ADD, ADD]
        tree = [L(0), L(1), MUL, L(0), SUB, L(1), DIV, L(2), SIN, L(2), ADD, ADD]
        assert np.array_equal(_out(prog, X, mode=mode), _out(tree, X, mode=mode),
                              equal_nan=True)

    def test_parser_reads_variables(self):
        nodes, consts = gcl.parse("LOAD a:0; COPY @2; LOAD b:1; ADD; PASTE @2; MUL;")
        assert list(nodes) == [L(0), V(COPY, 2), L(1), ADD, V(PASTE, 2), MUL]
        nodes, _ = gcl.parse("LOAD a:0; ARCSIN; ARCCOS; ARCTAN; TANH; TAN; CBRT; CUBE; "
                             "SIGN; SQUARE; LOAD b:1; POW;")
        assert list(nodes) == [L(0), ASIN, ACOS, ATAN, TANH, TAN, CBRT, CUBE, SIGN, SQUARE,
                               L(1), POW]


class TestMathCommands:
    def test_exact_values(self):
        X = np.array([[-27.0, 8.0, 3.0, -2.0, 0.0, 0.5]], np.float32)
        # glibc's cbrt is within an ulp, not correctly rounded (-27 gives
        # -3 - 2^-51)
        cb = _out([L(0), CBRT], X)
        assert np.allclose(cb, [-3.0, 2.0, 3.0 ** (1 / 3), -(2.0 ** (1 / 3)), 0.0,
                                0.5 ** (1 / 3)], rtol=4.5e-16, atol=0.0)
        assert list(_out([L(0), CUBE], X)) == [-19683.0, 512.0, 27.0, -8.0, 0.0, 0.125]
        assert list(_out([L(0), SQUARE], X)) == [729.0, 64.0, 9.0, 4.0, 0.0, 0.25]
        assert list(_out([L(0), SIGN], X)) == [27.0, -8.0, -3.0, 2.0, -0.0, -0.5]
        consts = np.array([2.0, 10.0, 9.0, 0.5, -8.0, 1 / 3, 0.0, -1.0], np.float32)
        one = np.zeros((1, 1), np.float32)
        assert _out([C(0), C(1), POW], one, consts)[0] == 1024.0
        assert _out([C(2), C(3), POW], one, consts)[0] == 3.0
        assert math.isnan(_out([C(4), C(5), POW], one, consts)[0])     # (-8)^(1/3)
        assert _out([C(6), C(7), POW], one, consts)[0] == math.inf     # 0^-1
        assert _out([C(4), C(6), POW], one, consts)[0] == 1.0          # x^0

    def test_inverse_trig_closed_forms(self):
        X = np.array([[1.0, -1.0, 0.0, 0.5, -0.5]], np.float32)
        assert np.allclose(_out([L(0), ASIN], X), [math.pi / 2, -math.pi / 2, 0.0,
                                                  math.pi / 6, -math.pi / 6], rtol=1e-15)
        assert np.allclose(_out([L(0), ACOS], X), [0.0, math.pi, math.pi / 2, math.pi / 3,
                                                  2 * math.pi / 3], rtol=1e-15, atol=1e-300)
        assert np.allclose(_out([L(0), ATAN], X)[:3], [math.pi / 4, -math.pi / 4, 0.0],
                           rtol=1e-15)
        # outside the domain: NaN (unprotected), so the program's fitness is +inf
        Xd = np.array([[1.5, -1.0000001]], np.float32)
        for op in (ASIN, ACOS):
            assert np.isnan(_out([L(0), op], Xd)).all()
        F, _, st = oracle.fitness(np.array([L(0), ASIN], np.uint32), np.array([0, 2]),
                                  np.zeros(1, np.float32), Xd, np.zeros(2, np.float32), 0.0,
                                  MASK)
        assert st[0] == 0 and F[0] == math.inf

    def test_identities_on_random_inputs(self):
        X = _X(n=2001, lo=-1.5, hi=1.5)
        x = X[0].astype(np.float64)
        s, c = np.sin(x), np.cos(x)
        assert np.allclose(_out([L(0), TAN], X), s / c, rtol=1e-14)
        assert np.allclose(_out([L(0), SIN, ASIN], X), x, rtol=1e-13, atol=1e-15)
        assert np.allclose(_out([L(0), COS, ACOS], X), np.abs(x), rtol=1e-13, atol=1e-7)
        assert np.allclose(_out([L(0), TAN, ATAN], X), x, rtol=1e-14, atol=1e-15)
        em = np.expm1(2 * x)
        assert np.allclose(_out([L(0), TANH], X), em / (em + 2), rtol=1e-14, atol=1e-300)
        assert np.allclose(_out([L(0), CBRT, CUBE], X), x, rtol=2e-15, atol=1e-300)
        ax = np.abs(x) + 0.25
        Xp = np.stack([ax, X[1].astype(np.float64)]).astype(np.float32)
        a, b = Xp[0].astype(np.float64), Xp[1].astype(np.float64)
        assert np.allclose(_out([L(0), L(1), POW], Xp), np.exp(b * np.log(a)), rtol=1e-14)
        assert np.array_equal(_out([L(0), CUBE], Xp), a * a * a)

    def test_raw_and_protected_square_root(self):
        X = np.array([[4.0, -4.0, 0.0]], np.float32)
        assert list(_out([L(0), SQRT], X)) == [2.0, 2.0, 0.0]
        r = _out([L(0), SQRT_RAW], X)
        assert r[0] == 2.0 and math.isnan(r[1]) and r[2] == 0.0

    def test_perturbed_modes_move_the_new_functions(self):
        # the certification modes nudge every elementary function result
        X = np.array([[0.3]], np.float32)
        for op in (CBRT, TAN, ASIN, ACOS, ATAN, TANH, SQRT_RAW):
            up = _out([L(0), op], X, mode=oracle.M32E_UP)[0]
            e = _out([L(0), op], X, mode=oracle.M32E)[0]
            assert up == float(np.nextafter(np.float32(e), np.float32(np.inf))), op


def _brute_status(prog, n_vars=1, n_consts=1):
    """Validity written out independently: the stack as a list of markers,
    variables as a set of names."""
    stack, held, peak = [], set(), 0
    for w in prog:
        op, arg = w & 0xFF, w >> 8
        need = {LOAD: 0, CONST: 0, PASTE: 0, DUP: 1, DEL: 1, COPY: 1, SWAP: 2, ADD: 2,
                SUB: 2, MUL: 2, DIV: 2, POW: 2}.get(op, 1)
        if op == LOAD and arg >= n_vars:
            return oracle.ST_BAD_VAR, 0
        if op == CONST and arg >= n_consts:
            return oracle.ST_BAD_CONST, 0
        if len(stack) < need:
            return oracle.ST_UNDERFLOW, 0
        if op == COPY:
            if arg >= 16 or arg in held:
                return oracle.ST_BAD_PAIR, 0
            held.add(arg)
        elif op == PASTE:
            if arg >= 16 or arg not in held:
                return oracle.ST_BAD_PAIR, 0
            held.discard(arg)
            stack.append(1)
        elif op in (LOAD, CONST, DUP):
            stack.append(1)
        elif op == DEL or need == 2 and op != SWAP:
            stack.pop()
        if len(stack) + len(held) > 32:
            return oracle.ST_TOO_DEEP, 0
        peak = max(peak, len(stack) + len(held))
    if len(stack) != 1:
        return oracle.ST_FINAL_DEPTH, peak
    if held:
        return oracle.ST_BAD_PAIR, peak
    return oracle.ST_VALID, peak


class TestValidity:
    def test_hand_made_cases(self):
        cases = [([L(0), V(COPY, 0)], oracle.ST_BAD_PAIR),
                 ([V(PASTE, 0)], oracle.ST_BAD_PAIR),
                 ([L(0), V(COPY, 16), V(PASTE, 16), ADD], oracle.ST_BAD_PAIR),
                 ([L(0), V(COPY, 1), V(COPY, 1), V(PASTE, 1), ADD], oracle.ST_BAD_PAIR),
                 ([L(0), V(COPY, 1), V(PASTE, 1), V(PASTE, 1), ADD, ADD], oracle.ST_BAD_PAIR),
                 ([DUP], oracle.ST_UNDERFLOW), ([L(0), SWAP], oracle.ST_UNDERFLOW),
                 ([L(0), DEL], oracle.ST_FINAL_DEPTH),
                 ([L(0), V(COPY, 2), V(PASTE, 2), MUL], oracle.ST_VALID)]
        for prog, want in cases:
            st, _ = oracle.validate(np.array(prog, np.uint32), np.array([0, len(prog)]), 1, 1,
                                    MASK)
            assert st[0] == want, (prog, st[0])

    def test_variables_share_the_32_cells(self):
        # 16 live variables and 16 stack elements fill the 32 cells; one more
        # element does not fit
        prog = [L(0)] + [V(COPY, k) for k in range(16)] + [L(0)] * 15
        tail = [ADD] * 15 + [V(PASTE, k) for k in range(16)] + [ADD] * 16
        st, md = oracle.validate(np.array(prog + tail, np.uint32),
                                 np.array([0, len(prog + tail)]), 1, 1, MASK)
        assert st[0] == oracle.ST_VALID and md[0] == 32
        prog2 = prog + [L(0)] + [ADD] + tail
        st, _ = oracle.validate(np.array(prog2, np.uint32), np.array([0, len(prog2)]), 1, 1,
                                MASK)
        assert st[0] == oracle.ST_TOO_DEEP

    def test_brute_force_short_programs(self):
        alphabet = [L(0), C(0), SIN, ADD, POW, DUP, SWAP, DEL, V(COPY, 0), V(PASTE, 0),
                    V(COPY, 1), V(PASTE, 1)]
        progs = [list(t) for n in range(1, 6) for t in itertools.product(alphabet, repeat=n)]
        lens = [len(p) for p in progs]
        nodes = np.array([w for p in progs for w in p], np.uint32)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        st, md = oracle.validate(nodes, off, 1, 1, MASK)
        n_valid = 0
        for i, p in enumerate(progs):
            want, peak = _brute_status(p)
            assert st[i] == want, (p, st[i], want)
            if want == oracle.ST_VALID:
                assert md[i] == peak
                n_valid += 1
        assert n_valid > 500                 # 814 with this alphabet
