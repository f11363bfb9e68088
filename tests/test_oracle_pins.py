"""Pins of the fp64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them re-types the oracle's formula:
values come from hand computation, the paper's printed genomes, exact
rational arithmetic, generating-function counts, an independent tree
evaluator, or invariants.
"""
import math
import os
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import (ABS, ADD, CONST, COS, DIV, EXP, LOAD, LOG, MUL, SIN, SQRT,
                    SUB, M32E, M32E_DN, M32E_UP, M64)
from oracle import gcl, tree_eval

HERE = os.path.dirname(os.path.abspath(__file__))
F32MAX = float(np.finfo(np.float32).max)
THETA = float(np.float32(0.001))


def f32(v):
    return float(np.float32(v))


def prog(*toks):
    """Tiny assembler: ints are opcodes; ('x', k) LOAD k; ('c', j) CONST j."""
    out = []
    for t in toks:
        if isinstance(t, tuple):
            out.append((LOAD if t[0] == "x" else CONST) | (t[1] << 8))
        else:
            out.append(t)
    return np.array(out, np.uint32)


def one_case(p, xs, consts=(), mode=M64):
    X = np.array(xs, np.float32).reshape(-1, 1)
    c = np.array(consts, np.float32)
    return oracle.program_outputs(p, c, X, mode=mode, allowed_mask=oracle.MASK_GCL)[0]


def fit1(p, X, y, consts=(), tax=0.0, mode=M64):
    p = np.asarray(p, np.uint32)
    F, mse, st = oracle.fitness(p, [0, p.size], np.array(consts, np.float32),
                                np.asarray(X, np.float32), np.asarray(y, np.float32),
                                tax, allowed_mask=oracle.MASK_GCL, mode=mode)
    assert st[0] == 0
    return F[0], mse[0]


# ---------------------------------------------------------------- P1
class TestHandComputed:
    """P1: op semantics, operand order and protections (GCL command table;
    protected-operator readings)."""

    def test_sub_is_second_minus_top(self):
        assert one_case(prog(("x", 0), ("x", 1), SUB), [3, 1]) == 2.0
        assert one_case(prog(("x", 1), ("x", 0), SUB), [3, 1]) == -2.0

    def test_div_is_second_over_top(self):
        assert one_case(prog(("c", 0), ("c", 1), DIV), [0], [2, 4]) == 0.5

    @pytest.mark.parametrize("c", [0.0, -0.0, THETA, -THETA])
    def test_protected_div_at_and_below_theta(self, c):
        assert one_case(prog(("x", 0), ("c", 0), DIV), [7], [c]) == 1.0

    def test_div_just_above_theta(self):
        c = np.nextafter(np.float32(THETA), np.float32(1))
        assert one_case(prog(("x", 0), ("c", 0), DIV), [7], [c]) == 7.0 / float(c)
        c = f32(0.0011)
        assert one_case(prog(("x", 0), ("c", 0), DIV), [3], [c]) == 3.0 / c

    def test_div_nan_divisor_stays_nan(self):
        # exp(89) - exp(89) = inf - inf = NaN as divisor: not laundered to 1
        p = prog(("x", 0), ("x", 1), EXP, ("x", 1), EXP, SUB, DIV)
        assert math.isnan(one_case(p, [5, 89]))

    def test_negative_zero_constant(self):
        v = one_case(prog(("c", 0), ("x", 1), ADD), [0, 2.5], [-0.0])
        assert v == 2.5
        v = one_case(prog(("c", 0),), [0], [-0.0])
        assert v == 0.0 and math.copysign(1, v) < 0

    def test_protected_log(self):
        assert one_case(prog(("x", 0), LOG), [0]) == 0.0
        assert one_case(prog(("x", 0), LOG), [THETA]) == 0.0
        assert one_case(prog(("x", 0), LOG), [-THETA]) == 0.0
        e = f32(-math.e)
        assert abs(one_case(prog(("x", 0), LOG), [e]) - 1.0) < 1e-7
        assert one_case(prog(("x", 0), LOG), [1.0]) == 0.0
        assert one_case(prog(("x", 0), EXP, LOG), [89]) == math.inf

    def test_protected_sqrt(self):
        assert one_case(prog(("x", 0), SQRT), [-4]) == 2.0
        assert one_case(prog(("x", 0), SQRT), [9]) == 3.0

    def test_unary_basics(self):
        assert one_case(prog(("x", 0), SIN), [0]) == 0.0
        assert one_case(prog(("x", 0), COS), [0]) == 1.0
        assert one_case(prog(("x", 0), EXP), [0]) == 1.0
        assert one_case(prog(("x", 0), ABS), [-3]) == 3.0

    def test_exp_overflow_is_worst(self):
        X = np.array([[89.0]], np.float32)
        F, _ = fit1(prog(("x", 0), EXP), X, [0.0])
        assert F == math.inf

    def test_exp88_finite_but_mse_overflows(self):
        X = np.array([[88.0]], np.float32)
        v = one_case(prog(("x", 0), EXP), [88])
        assert math.isfinite(v) and 1.6e38 < v < F32MAX
        F, mse = fit1(prog(("x", 0), EXP), X, [0.0])
        assert mse > F32MAX and F == math.inf

    def test_inf_over_inf_is_worst(self):
        X = np.array([[89.0]], np.float32)
        p = prog(("x", 0), EXP, ("x", 0), EXP, DIV)
        assert math.isnan(one_case(p, [89]))
        assert fit1(p, X, [0.0])[0] == math.inf

    def test_sin_of_inf_is_nan(self):
        assert math.isnan(one_case(prog(("x", 0), EXP, SIN), [89]))


class TestOverflowEmulation:
    """R(v): an fp64 value whose fp32 rounding overflows becomes +-inf.
    The edge is pinned against numpy's IEEE fp64->fp32 conversion."""

    def test_edge_matches_numpy_cast(self):
        edge = math.ldexp(2 - 2 ** -24, 127)        # FLT_MAX + 2^103
        with np.errstate(over="ignore"):
            assert np.isinf(np.float32(edge))
            assert not np.isinf(np.float32(np.nextafter(edge, 0)))
        big = f32(F32MAX)
        # FLT_MAX + 2^103 is exactly the edge in fp64 -> inf
        assert one_case(prog(("c", 0), ("c", 1), ADD), [0], [big, 2.0 ** 103]) == math.inf
        assert one_case(prog(("c", 0), ("c", 1), ADD), [0], [-big, -2.0 ** 103]) == -math.inf
        # FLT_MAX + 2^102 stays finite (and is not rounded in M64)
        v = one_case(prog(("c", 0), ("c", 1), ADD), [0], [big, 2.0 ** 102])
        assert v == big + 2.0 ** 102
        # ... but M32E rounds it to FLT_MAX
        v = one_case(prog(("c", 0), ("c", 1), ADD), [0], [big, 2.0 ** 102], mode=M32E)
        assert v == big

    def test_square_overflow(self):
        assert one_case(prog(("x", 0), ("x", 0), MUL), [2e19]) == math.inf
        assert math.isfinite(one_case(prog(("x", 0), ("x", 0), MUL), [1.8e19]))

    def test_m32e_rounds_each_op(self):
        p = prog(("c", 0), ("c", 1), ADD)
        assert one_case(p, [0], [1.0, 2.0 ** -30]) == 1.0 + 2.0 ** -30
        assert one_case(p, [0], [1.0, 2.0 ** -30], mode=M32E) == 1.0

    def test_perturbed_modes_move_one_ulp(self):
        p = prog(("x", 0), SIN)
        base = one_case(p, [0.5], mode=M32E)
        up = one_case(p, [0.5], mode=M32E_UP)
        dn = one_case(p, [0.5], mode=M32E_DN)
        assert up == float(np.nextafter(np.float32(base), np.float32(2)))
        assert dn == float(np.nextafter(np.float32(base), np.float32(-2)))
        # non-transcendental ops are not perturbed
        q = prog(("x", 0), ("x", 0), ADD)
        assert one_case(q, [0.5], mode=M32E_UP) == 1.0

    def test_random_mode_stays_within_two_ulps(self):
        X = np.linspace(-3, 3, 512).astype(np.float32).reshape(1, -1)
        p = prog(("x", 0), EXP)
        base = oracle.program_outputs(p, [], X, mode=M32E).astype(np.float32)
        seen = set()
        for seed in range(3):
            v = oracle.program_outputs(p, [], X, mode=oracle.M32E_RAND + seed).astype(np.float32)
            d = (v.view(np.int32).astype(np.int64) - base.view(np.int32).astype(np.int64))
            assert np.all(np.abs(d) <= 2)
            seen.update(np.unique(d).tolist())
            again = oracle.program_outputs(p, [], X, mode=oracle.M32E_RAND + seed)
            assert np.array_equal(again, v.astype(np.float64))      # deterministic
        assert seen == {-2, -1, 0, 1, 2}


class TestValidator:
    """Stack discipline (RPN; 32-element limit; final depth 1)."""

    def chk(self, p, n_consts=1, n_vars=2, mask=oracle.MASK_BENCH):
        p = np.asarray(p, np.uint32)
        st, md = oracle.validate(p, [0, p.size], n_consts, n_vars, mask)
        return st[0], md[0]

    def test_valid(self):
        assert self.chk(prog(("x", 0), ("x", 1), ADD)) == (0, 2)

    def test_codes(self):
        assert self.chk(np.zeros(0, np.uint32))[0] == oracle.ST_EMPTY
        assert self.chk(prog(("x", 0), 200))[0] == oracle.ST_BAD_OP
        assert self.chk(prog(("x", 0), oracle.DUP, ADD))[0] == oracle.ST_BAD_OP
        assert self.chk(prog(("x", 2)))[0] == oracle.ST_BAD_VAR
        assert self.chk(prog(("c", 1)))[0] == oracle.ST_BAD_CONST
        assert self.chk(prog(("x", 0), ADD))[0] == oracle.ST_UNDERFLOW
        assert self.chk(prog(SIN))[0] == oracle.ST_UNDERFLOW
        assert self.chk(prog(("x", 0), ("x", 1)))[0] == oracle.ST_FINAL_DEPTH

    def test_depth_limit(self):
        ok = prog(*([("x", 0)] * 32 + [ADD] * 31))
        assert self.chk(ok) == (0, 32)
        deep = prog(*([("x", 0)] * 33 + [ADD] * 32))
        assert self.chk(deep)[0] == oracle.ST_TOO_DEEP

    def test_disallowed_op(self):
        mask = oracle.MASK_BENCH & ~(1 << SIN)
        assert self.chk(prog(("x", 0), SIN), mask=mask)[0] == oracle.ST_BAD_OP


# ---------------------------------------------------------------- P2
def _paper_genomes():
    out = []
    with open(os.path.join(HERE, "golden", "paper_genomes.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, text = line.split("|", 1)
            out.append((int(n), text.strip()))
    return out


def _quadratic_data(n=512, seed=7):
    rng = np.random.default_rng(seed)
    a = (rng.uniform(0.5, 2.0, 4 * n) * rng.choice([-1, 1], 4 * n)).astype(np.float32)
    b = rng.uniform(-5, 5, 4 * n).astype(np.float32)
    c = rng.uniform(-5, 5, 4 * n).astype(np.float32)
    a64, b64, c64 = (v.astype(np.float64) for v in (a, b, c))
    keep = (b64 * b64 - 4 * a64 * c64) >= 0
    X = np.stack([a[keep][:n], b[keep][:n], c[keep][:n]])
    return X


class TestPaperGenomes:
    """P2: the two genomes printed in the paper's console example."""

    def test_printed_lengths(self):
        for n, text in _paper_genomes():
            nodes, consts = gcl.parse(text)
            assert nodes.size == n

    def test_quadratic_root(self):
        X = _quadratic_data()
        a, b, c = (X[i].astype(np.float64) for i in range(3))
        root = (-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)
        scale = (np.abs(b) + np.sqrt(np.abs(b * b - 4 * a * c))) / np.abs(a)
        for n, text in _paper_genomes():
            nodes, consts = gcl.parse(text)
            out = oracle.program_outputs(nodes, consts, X, allowed_mask=oracle.MASK_GCL)
            assert np.all(np.abs(out - root) <= 1e-12 * scale + 1e-300)
            # the paper's "perfect" rule: every case within 0.1%
            assert np.all(np.abs(out - root) <= 1e-3 * np.abs(root) + 1e-9 * scale)

    def test_tax_counts_every_node(self):
        X = _quadratic_data(64)
        for n, text in _paper_genomes():
            nodes, consts = gcl.parse(text)
            y = np.zeros(64, np.float32)
            F0, _ = fit1(nodes, X, y, consts, tax=0.0)
            F1, _ = fit1(nodes, X, y, consts, tax=1e-3)
            assert abs((F1 - F0) - 1e-3 * n) <= 4 * np.spacing(F1)

    def test_restricted_opset_translation(self):
        # the same root with only {LOAD, CONST, +, -, *, /, sqrt}
        X = _quadratic_data()
        a, b, c = (X[i].astype(np.float64) for i in range(3))
        root = (-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)
        scale = (np.abs(b) + np.sqrt(np.abs(b * b - 4 * a * c))) / np.abs(a)
        p = prog(("x", 1), ("x", 1), MUL, ("c", 0), ("x", 0), MUL, ("x", 2), MUL, SUB,
                 SQRT, ("x", 1), SUB, ("x", 0), DIV, ("c", 1), MUL)
        out = oracle.program_outputs(p, np.array([4, 0.5], np.float32), X)
        assert np.all(np.abs(out - root) <= 1e-12 * scale)


# ---------------------------------------------------------------- P3
def _exact_mse(vals, y):
    """Exact rational mean of squared residuals."""
    n = len(y)
    s = sum((Fraction(float(v)) - Fraction(float(t))) ** 2 for v, t in zip(vals, y))
    return s / n


class TestClosedForms:
    """P3: programs whose fitness has a closed form."""

    def setup_method(self):
        rng = np.random.default_rng(11)
        self.X = rng.uniform(-3, 3, (3, 1000)).astype(np.float32)

    def test_variable_equal_to_target(self):
        for k in range(3):
            F, mse = fit1(prog(("x", k)), self.X, self.X[k], tax=1e-3)
            assert mse == 0.0 and F == 1e-3

    def test_constant_program(self):
        y = self.X[1]
        c = f32(0.37)
        F, mse = fit1(prog(("c", 0)), self.X, y, [c])
        ex = _exact_mse([c] * y.size, y)
        assert abs(mse - float(ex)) <= 1e-13 * float(ex)

    def test_protected_zero_division(self):
        y = self.X[2]
        F, mse = fit1(prog(("x", 0), ("c", 0), DIV), self.X, y, [0.0])
        ex = _exact_mse([1.0] * y.size, y)
        assert abs(mse - float(ex)) <= 1e-13 * float(ex)

    def test_self_difference(self):
        y = self.X[2]
        F, mse = fit1(prog(("x", 0), ("x", 0), SUB), self.X, y)
        ex = _exact_mse([0.0] * y.size, y)
        assert abs(mse - float(ex)) <= 1e-13 * float(ex)


class TestInvalidTargets:
    """P3b: targets that are NaN or +-inf (Sec. "Fitness Functions": invalid
    values in the model output or the dataset are handled, not removed; as
    in Eq. 2, a case where output and target are both invalid is a matched
    pair, a case where exactly one is invalid is a mismatch).  Reading: a
    matched pair adds no error, a mismatch makes F = +inf, and the mean
    divides by all n cases.  Every value here is computed by hand."""

    INF, NAN = float("inf"), float("nan")

    def _fit(self, p, xs, y, consts=(), tax=0.0):
        X = np.array(xs, np.float32).reshape(1, -1)
        return fit1(p, X, np.array(y, np.float32), consts, tax)

    def test_matched_pairs_add_nothing(self):
        # outputs [inf, 1, 2], targets [nan, 1, 5]: case 0 matched (both
        # invalid), case 1 error 0, case 2 error (2 - 5)^2 = 9: MSE = 9/3
        F, mse = self._fit(prog(("x", 0)), [self.INF, 1.0, 2.0], [self.NAN, 1.0, 5.0],
                           tax=0.5)
        assert mse == 3.0 and F == 3.5

    @pytest.mark.parametrize("yv", [float("nan"), float("inf"), -float("inf")])
    def test_finite_output_against_invalid_target_is_worst(self, yv):
        F, _ = self._fit(prog(("x", 0)), [0.0, 1.0, 2.0], [yv, 1.0, 2.0])
        assert F == math.inf

    def test_invalid_output_against_finite_target_is_worst(self):
        # exp(89) overflows fp32: +inf against a finite target
        F, _ = self._fit(prog(("x", 0), EXP), [89.0, 0.0], [1.0, 1.0])
        assert F == math.inf

    def test_any_pairing_of_nan_and_inf_is_matched(self):
        # exp(89) = +inf against -inf, sin(inf) = NaN against +inf, and
        # 0 * inf = NaN against NaN are all matched; the last case adds
        # (1 - 3)^2 = 4 out of 4 cases
        p_exp = prog(("x", 0), EXP)
        F, mse = self._fit(p_exp, [89.0, 89.0, 0.0, 0.0],
                           [-self.INF, self.NAN, 1.0, 3.0])
        assert mse == 1.0 and F == 1.0
        F, mse = self._fit(prog(("x", 0), SIN), [self.INF, 0.5], [self.INF, f32(math.sin(0.5))])
        assert mse == (f32(math.sin(0.5)) - math.sin(f32(0.5))) ** 2 / 2

    def test_all_cases_matched_gives_tax_only(self):
        F, mse = self._fit(prog(("x", 0), ("x", 0), MUL), [self.INF, self.NAN],
                           [self.NAN, -self.INF], tax=0.25)
        assert mse == 0.0 and F == 0.75

    def test_valid_program_never_nan(self):
        # every mixture of finite and invalid targets gives a number or +inf
        rng = np.random.default_rng(3)
        X = rng.uniform(-2, 2, (2, 64)).astype(np.float32)
        X[0, ::7] = np.inf
        y = rng.uniform(-2, 2, 64).astype(np.float32)
        y[::5] = np.nan
        y[1::9] = -np.inf
        for toks in [(("x", 0),), (("x", 1),), (("x", 0), ("x", 1), ADD),
                     (("x", 0), EXP), (("x", 1), LOG)]:
            F, _ = fit1(prog(*toks), X, y)
            assert not math.isnan(F)


# ---------------------------------------------------------------- P4
def _int_tree_value(tree, xs):
    """Exact integer evaluation of a {+,-,*} tree: (value, largest |value| of
    any subtree)."""
    k = tree[0]
    if k == "x":
        v = int(xs[tree[1]])
        return v, abs(v)
    if k == "c":
        v = int(tree[1])
        return v, abs(v)
    (a, ma), (b, mb) = _int_tree_value(tree[2], xs), _int_tree_value(tree[3], xs)
    v = {ADD: a + b, SUB: a - b, MUL: a * b}[tree[1]]
    return v, max(ma, mb, abs(v))


def exact_family(n_programs=400, n_cases=64, seed=5):
    """Small-integer programs over {+,-,*} (n a power of two)."""
    from paper_2607_06731_amd import synth
    rng = np.random.default_rng(seed)
    lens = 2 * rng.integers(1, 8, n_programs) + 1
    pop = synth.sample_programs(rng, lens, 2, unary=(), binary=(ADD, SUB, MUL))
    pop.consts[:] = rng.integers(-3, 4, pop.consts.size).astype(np.float32)
    X = rng.integers(-4, 5, (2, n_cases)).astype(np.float32)
    y = rng.integers(-8, 9, n_cases).astype(np.float32)
    return pop, X, y


class TestExactFamily:
    """P4: integer data and {+,-,*}: exact Python-integer evaluation of the
    parsed tree, exact mean; the oracle must agree bit for bit whenever the
    exact value is representable."""

    def test_bit_exact_against_integers(self):
        pop, X, y = exact_family()
        F, mse, st = oracle.fitness(pop.nodes, pop.offsets, pop.consts, X, y, 0.0,
                                    allowed_mask=oracle.MASK_BENCH)
        assert np.all(st == 0)
        checked = 0
        for p in range(pop.n_programs):
            nodes = pop.nodes[pop.offsets[p]:pop.offsets[p + 1]]
            tree = tree_eval.parse(nodes, pop.consts, 2)
            res = [_int_tree_value(tree, X[:, i]) for i in range(X.shape[1])]
            vals = [v for v, _ in res]
            if max(m for _, m in res) >= 2 ** 24:
                continue
            s = sum((v - int(t)) ** 2 for v, t in zip(vals, y))
            if s >= 2 ** 52:
                continue
            assert mse[p] == float(Fraction(s, X.shape[1])), p
            checked += 1
        assert checked > 300

    def test_const_index_family(self):
        # program p = CONST p with consts[p] = p mod 4096 and y = 0:
        # MSE = (p mod 4096)^2 exactly, for a million programs
        P = 1_000_000
        nodes = (CONST | (np.arange(P, dtype=np.uint32) << 8)).astype(np.uint32)
        offsets = np.arange(P + 1, dtype=np.int64)
        consts = (np.arange(P) % 4096).astype(np.float32)
        X = np.zeros((1, 4), np.float32)
        y = np.zeros(4, np.float32)
        F, mse, st = oracle.fitness(nodes, offsets, consts, X, y, 0.0)
        ex = (np.arange(P) % 4096).astype(np.float64) ** 2
        assert np.array_equal(F, ex)


# ---------------------------------------------------------------- P5
SPECIAL = [0.0, THETA, -THETA, 0.0011, -0.0011, 1.0, -1.0, 3.0, -3.0, 44.0, 88.0, 89.0, -89.0]
ALPHABET = ([LOAD | (0 << 8), LOAD | (1 << 8), CONST | (0 << 8)]
            + [SIN, COS, EXP, LOG, SQRT, ABS] + [ADD, SUB, MUL, DIV])


def gf_counts(max_len):
    """Coefficients of T(z) = 3z + 6zT + 4zT^2: number of valid programs per
    length for 3 leaves, 6 unary and 4 binary ops."""
    a = [0] * (max_len + 1)
    for n in range(1, max_len + 1):
        a[n] = (3 if n == 1 else 0) + 6 * a[n - 1] + \
            4 * sum(a[i] * a[n - 1 - i] for i in range(1, n - 1))
    return a


def brute_force_programs(max_len=5):
    """Every token sequence of length <= max_len over the alphabet."""
    import itertools
    seqs = []
    for L in range(1, max_len + 1):
        for t in itertools.product(ALPHABET, repeat=L):
            seqs.append(t)
    return seqs


@pytest.fixture(scope="module")
def brute():
    seqs = brute_force_programs()
    lens = np.array([len(s) for s in seqs], np.int64)
    offsets = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    nodes = np.array([t for s in seqs for t in s], np.uint32)
    st, md = oracle.validate(nodes, offsets, 1, 2, oracle.MASK_BENCH)
    return seqs, nodes, offsets, st


class TestBruteForce:
    """P5: all programs of length <= 5 over {x0, x1, c} and the benchmark
    ops."""

    def test_gf_counts(self):
        assert gf_counts(5)[1:] == [3, 18, 144, 1296, 12528]

    def test_validator_accepts_exactly_the_gf_count(self, brute):
        seqs, nodes, offsets, st = brute
        lens = np.diff(offsets)
        counts = [int(np.sum((st == 0) & (lens == L))) for L in range(1, 6)]
        assert counts == gf_counts(5)[1:]
        assert int(np.sum(st == 0)) == 13989

    def test_tree_parser_agrees_on_accept_reject(self, brute):
        seqs, nodes, offsets, st = brute
        consts = [0.5]
        for s, code in zip(seqs, st):
            try:
                tree_eval.parse(s, consts, 2)
                ok = True
            except tree_eval.Invalid:
                ok = False
            assert ok == (code == 0)

    def test_values_match_tree_evaluator(self, brute):
        seqs, nodes, offsets, st = brute
        consts = np.array([-0.0011], np.float32)
        x0 = np.repeat(np.array(SPECIAL, np.float32), 5)
        x1 = np.tile(np.array([0.0, -THETA, 1.0, 44.0, -89.0], np.float32), len(SPECIAL))
        X = np.stack([x0, x1]).astype(np.float32)
        valid = np.nonzero(st == 0)[0]
        for p in valid:
            s = seqs[p]
            ours = oracle.program_outputs(np.array(s, np.uint32), consts, X)
            ref = tree_eval.outputs(s, consts, X)
            same = (ours == ref) | (np.isnan(ours) & np.isnan(ref))
            assert same.all(), (s, ours[~same], ref[~same])


# ---------------------------------------------------------------- P6
class TestInvariants:
    """P6: commutativity, case permutation / duplication, tax linearity."""

    def setup_method(self):
        from paper_2607_06731_amd import synth
        self.w = synth.make_workload("generation", n_programs=300, n_cases=512)

    def test_commutative_ops_bitwise(self):
        pop = self.w.pop
        X = self.w.data.X
        for p in range(0, 40, 2):
            a = pop.nodes[pop.offsets[p]:pop.offsets[p + 1]]
            b = pop.nodes[pop.offsets[p + 1]:pop.offsets[p + 2]]
            for op in (ADD, MUL):
                ab = np.concatenate([a, b, [op]]).astype(np.uint32)
                ba = np.concatenate([b, a, [op]]).astype(np.uint32)
                va = oracle.program_outputs(ab, pop.consts, X)
                vb = oracle.program_outputs(ba, pop.consts, X)
                same = (va == vb) | (np.isnan(va) & np.isnan(vb))
                assert same.all()

    def test_case_permutation_and_duplication(self):
        w = self.w
        F, _, _ = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts,
                                 w.data.X, w.data.y, w.tax, w.allowed_mask)
        perm = np.random.default_rng(3).permutation(w.data.n_cases)
        Fp, _, _ = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts,
                                  w.data.X[:, perm], w.data.y[perm], w.tax, w.allowed_mask)
        Fd, _, _ = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts,
                                  np.concatenate([w.data.X, w.data.X], 1),
                                  np.concatenate([w.data.y, w.data.y]), w.tax, w.allowed_mask)
        fin = np.isfinite(F)
        assert np.array_equal(fin, np.isfinite(Fp)) and np.array_equal(fin, np.isfinite(Fd))
        assert np.all(np.abs(Fp[fin] - F[fin]) <= 1e-12 * np.abs(F[fin]))
        assert np.all(np.abs(Fd[fin] - F[fin]) <= 1e-12 * np.abs(F[fin]))

    def test_tax_is_linear_in_length(self):
        w = self.w
        F0, _, _ = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts,
                                  w.data.X, w.data.y, 0.0, w.allowed_mask)
        F1, _, _ = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts,
                                  w.data.X, w.data.y, 0.25, w.allowed_mask)
        fin = np.isfinite(F0)
        assert np.array_equal(fin, np.isfinite(F1))
        lens = w.pop.lengths[fin]
        F0, F1 = F0[fin], F1[fin]
        assert np.all(np.abs((F1 - F0) - 0.25 * lens) <= 2 * np.spacing(F1))


# ---------------------------------------------------------------- P7
class TestPrecisionPin:
    """P7: a million cases with an exactly known MSE."""

    def test_million_case_exact_mean(self):
        n, m, h = 1 << 20, 1024, 16.0
        i = np.arange(n)
        y = (h * ((i % m) - (m - 1) / 2.0)).astype(np.float32)
        assert np.array_equal(y.astype(np.float64), h * ((i % m) - (m - 1) / 2.0))
        X = np.zeros((1, n), np.float32)
        F, mse = fit1(prog(("c", 0)), X, y, [0.0])
        exact = Fraction(int(h) ** 2 * (m * m - 1), 12)
        assert mse == float(exact)


# ------------------------------------------------- P8: correlation fitness
def corr1(p, X, y, consts=(), M=1e4, mode=M64):
    p = np.asarray(p, np.uint32)
    s, r, st = oracle.correlation(p, [0, p.size], np.array(consts, np.float32),
                                  np.asarray(X, np.float32), np.asarray(y, np.float32), M,
                                  allowed_mask=oracle.MASK_GCL, mode=mode)
    assert st[0] == 0
    return s[0], r[0]


def _eq2(r, N, c1, c2, M):
    """Eq. 2 with r^4 = (r^2)^2."""
    return M * (r * r) ** 2 * (N - (c1 + c2)) - M * (c1 - c2)


class TestCorrelationPins:
    """The paper's correlation fitness (Eq. 1-2) pinned to exact rational
    arithmetic, to numpy's Pearson coefficient, to closed forms and to
    hand-counted invalid pairs."""

    def test_worked_example_exact(self):
        # f = x0 = 1, 2, 3, 4 against y = 2, 4, 5, 4: Sxy = 7/2, Sxx = 5,
        # Syy = 19/4, so r^2 = (49/4) / (95/4) = 49/95
        xs, ys = [1, 2, 3, 4], [2, 4, 5, 4]
        fb, yb = Fraction(sum(xs), 4), Fraction(sum(ys), 4)
        sxy = sum((Fraction(x) - fb) * (Fraction(y) - yb) for x, y in zip(xs, ys))
        sxx = sum((Fraction(x) - fb) ** 2 for x in xs)
        syy = sum((Fraction(y) - yb) ** 2 for y in ys)
        r2 = sxy * sxy / (sxx * syy)
        assert r2 == Fraction(49, 95)
        want = float(10000 * r2 * r2 * 4)
        s, r = corr1(prog(("x", 0)), [xs], ys)
        assert s == pytest.approx(want, rel=1e-14)
        assert r == pytest.approx(math.sqrt(49 / 95), rel=1e-14)

    @pytest.mark.parametrize("slope", [3.0, -0.25])
    def test_perfect_linear_relation_scores_M_N(self, slope):
        rng = np.random.default_rng(3)
        x = rng.uniform(-2, 2, 500).astype(np.float32)
        p = prog(("x", 0), ("c", 0), MUL, ("c", 1), SUB)     # slope * x - 0.5
        s, r = corr1(p, [x], x, consts=[slope, 0.5])
        assert abs(r) == pytest.approx(1.0, abs=1e-12)
        assert s == pytest.approx(1e4 * 500, rel=1e-10)

    def test_constant_output_or_target_scores_zero(self):
        x = np.linspace(-1, 1, 64, dtype=np.float32)
        s, r = corr1(prog(("c", 0)), [x], x, consts=[0.75])
        assert r == 0.0 and s == 0.0
        s, r = corr1(prog(("x", 0)), [x], np.full(64, 2.0, np.float32))
        assert r == 0.0 and s == 0.0

    def test_matches_numpy_pearson_on_random_programs(self):
        from paper_2607_06731_amd import synth
        w = synth.make_workload("generation", n_programs=60, n_cases=300)
        s, r, st = oracle.correlation(w.pop.nodes, w.pop.offsets, w.pop.consts,
                                      w.data.X, w.data.y, 1e4)
        y = w.data.y.astype(np.float64)
        checked = 0
        for p in range(60):
            f = oracle.program_outputs(w.pop.nodes[w.pop.offsets[p]:w.pop.offsets[p + 1]],
                                       w.pop.consts, w.data.X)
            ok = np.isfinite(f) & np.isfinite(y)
            c1 = int(np.sum(np.isfinite(f) != np.isfinite(y)))
            c2 = int(np.sum(~np.isfinite(f) & ~np.isfinite(y)))
            if ok.sum() >= 2 and np.std(f[ok]) > 0:
                rr = float(np.corrcoef(f[ok], y[ok])[0, 1])
                checked += 1
            else:
                rr = 0.0
            assert r[p] == pytest.approx(rr, rel=1e-9, abs=1e-12)
            assert s[p] == pytest.approx(_eq2(rr, 300, c1, c2, 1e4), rel=1e-8, abs=1e-6)
        assert checked >= 40

    def test_invalid_pairs_counted_on_both_sides(self):
        # x0 = 200 makes exp(x0) overflow to +inf; y = NaN marks an invalid
        # target.  Cases: 0-5 valid, 6-7 f invalid, 8-9 y invalid, 10 both.
        x = np.array([0.1, 0.5, -0.3, 0.9, 0.2, -0.7, 200, 200, 0.4, -0.2, 200], np.float32)
        y = np.array([1.0, 1.6, 0.8, 2.4, 1.2, 0.5, 3.0, 3.0, np.nan, np.nan, np.inf],
                     np.float32)
        s, r = corr1(prog(("x", 0), EXP), [x], y)
        f = np.exp(x[:6].astype(np.float64))
        rr = float(np.corrcoef(f, y[:6].astype(np.float64))[0, 1])
        assert r == pytest.approx(rr, rel=1e-12)
        # c1 = 4 (cases 6, 7, 8, 9), c2 = 1 (case 10), N = 11
        assert s == pytest.approx(_eq2(rr, 11, 4, 1, 1e4), rel=1e-12)
        p = prog(("x", 0), EXP)
        _, _, _, c1, c2 = oracle.correlation(p, [0, p.size], np.zeros(0, np.float32),
                                             x.reshape(1, -1), y, 1e4,
                                             allowed_mask=oracle.MASK_GCL, return_counts=True)
        assert (c1[0], c2[0]) == (4, 1)

    def test_all_outputs_invalid(self):
        x = np.full(8, 200, np.float32)
        s, r = corr1(prog(("x", 0), EXP), [x], np.ones(8, np.float32), M=5.0)
        assert r == 0.0 and s == -5.0 * 8

    def test_affine_invariance(self):
        from paper_2607_06731_amd import synth
        w = synth.make_workload("plain", n_programs=40, n_cases=256)
        base = w.pop
        c = np.concatenate([base.consts, np.array([2.5, 1.0], np.float32)]).astype(np.float32)
        ka, kb = base.consts.size, base.consts.size + 1
        progs = []
        for p in range(base.n_programs):
            q = base.nodes[base.offsets[p]:base.offsets[p + 1]]
            progs.append(np.concatenate([q, [CONST | (ka << 8), MUL, CONST | (kb << 8), ADD]]))
        nodes2 = np.concatenate(progs).astype(np.uint32)
        off2 = np.concatenate([[0], np.cumsum([len(q) for q in progs])]).astype(np.int64)
        s1, r1, _ = oracle.correlation(base.nodes, base.offsets, c, w.data.X, w.data.y, 1e4)
        s2, r2, _ = oracle.correlation(nodes2, off2, c, w.data.X, w.data.y, 1e4)
        fin = np.isfinite(s1) & (np.abs(r1) > 1e-3)
        assert fin.sum() >= 20
        assert np.allclose(s2[fin], s1[fin], rtol=1e-8)


# ---------------------------------------- P9: integer point-to-point reward
def _reward_of_pairs(o, y, power=1, M=1e4):
    """Reward of the identity program (output = x0 exactly) on pairs."""
    X = np.asarray(o, np.float32).reshape(1, -1)
    t, st = oracle.reward(np.array([LOAD], np.uint32), [0, 1], np.zeros(0, np.float32), X,
                          np.asarray(y, np.float32), M, power)
    assert st[0] == 0
    return t[0]


class TestRewardPins:
    """Eq. 5 (StdFitFunc) and its powers, pinned to hand-computed values."""

    def test_hand_computed_cases(self):
        M = 1e4
        # ratio 1/2 -> 5000; opposite signs -> 5000 - 10000/11 = 4090.9 -> 4091;
        # both zero -> M; equal -> M; zero against nonzero -> ratio 0 -> 0
        assert _reward_of_pairs([2], [4]) == 5000
        assert _reward_of_pairs([-2], [4]) == 4091
        assert _reward_of_pairs([0], [0]) == M
        assert _reward_of_pairs([3], [3]) == M
        assert _reward_of_pairs([0], [5]) == 0
        assert _reward_of_pairs([-0.0], [5]) == 0          # -0 has no sign penalty
        # invalid pairs: one side -> -M, both -> +M
        assert _reward_of_pairs([np.nan], [1]) == -M
        assert _reward_of_pairs([1], [np.inf]) == -M
        assert _reward_of_pairs([np.inf], [np.nan]) == M
        # the sum over cases
        assert _reward_of_pairs([2, -2, 0, 3, 0, np.nan, np.inf, 0.5],
                                [4, 4, 0, 3, 5, 1, np.nan, 1]) == 34091

    def test_powers(self):
        # ratio 1/2: ^2 -> 2500, ^3 -> 1250, ^8 -> 39.0625 -> 39;
        # with the sign penalty 39.0625 - 909.09 = -870.03 -> -870
        assert _reward_of_pairs([2], [4], 2) == 2500
        assert _reward_of_pairs([2], [4], 3) == 1250
        assert _reward_of_pairs([2], [4], 8) == 39
        assert _reward_of_pairs([-2], [4], 8) == -870

    def test_round_half_to_even(self):
        # M = 3, ratio 1/2 -> 1.5 -> 2; M = 5 -> 2.5 -> 2; M = 1 -> 0.5 -> 0
        assert _reward_of_pairs([1], [2], M=3.0) == 2
        assert _reward_of_pairs([1], [2], M=5.0) == 2
        assert _reward_of_pairs([1], [2], M=1.0) == 0

    def test_symmetry_and_scale_invariance(self):
        rng = np.random.default_rng(4)
        o = rng.standard_normal(200).astype(np.float32)
        y = rng.standard_normal(200).astype(np.float32)
        for p in (1, 2, 3, 8):
            a = _reward_of_pairs(o, y, p)
            assert _reward_of_pairs(y, o, p) == a            # min/max and sign symmetric
            assert _reward_of_pairs(o * 8, y * 8, p) == a    # powers of two keep the ratio
