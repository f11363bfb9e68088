"""GPU parity: the HIP path (through the C ABI) against the fp64 oracle.

Floating point: the gate of oracle.gate (1e-4 relative + 1e-12 absolute,
identical NaN/inf classes, fp32-certified exceptions counted).  Integer and
exact work (the exact-arithmetic family, constant indexing, validation
status codes) must be bit-exact.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import gate

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_06731_amd as gp
    gp.lib()        # raises if the HIP library is not built
    return gp


def _say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def _run(gp, pop_nodes, pop_offsets, consts, X, y, tax, mask, status=False):
    return gp.evaluate(pop_nodes, pop_offsets, consts, X, y, tax, mask, return_status=status)


def _gate(F, nodes, offsets, consts, X, y, tax, mask, label):
    rep = gate.check(F, nodes, offsets, consts, X, y, tax, mask)
    _say(label + ": " + rep.summary())
    assert rep.ok(), rep.failures[:10]
    return rep


# ------------------------------------------------------------ workloads
@pytest.mark.parametrize("name,P,n", [("plain", None, None), ("generation", 4000, None),
                                      ("uneven", 3000, 4000), ("precision", 48, 1 << 20),
                                      ("generation", 2000, 1025), ("generation", 2000, 7)])
def test_workload_parity(name, P, n):
    gp = _need_gpu()
    from paper_2607_06731_amd import synth
    w = synth.make_workload(name, n_programs=P, n_cases=n)
    label = "%s P=%d n=%d" % (name, w.pop.n_programs, w.data.n_cases)
    _say(label)
    F = _run(gp, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
             w.allowed_mask)
    _gate(F, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
          w.allowed_mask, label)


@pytest.mark.parametrize("n", [4096, 1025])
@pytest.mark.parametrize("matched", [False, True])
def test_invalid_targets_parity(n, matched):
    """3% of the targets NaN, +inf or -inf (Sec. "Fitness Functions": invalid
    values in the dataset are handled, not removed): matched invalid pairs
    add nothing, a mismatched case gives +inf; the gate separates NaN
    (structurally invalid) from +inf, and no valid program comes out NaN.

    Scattered invalid targets meet finite outputs, so every valid program
    scores +inf.  With ``matched``, every input of those cases is NaN too:
    a program that reads a variable outputs NaN there (every op propagates
    NaN), the pairs match and its score stays finite; a program of
    constants alone mismatches and scores +inf."""
    gp = _need_gpu()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=3000, n_cases=n)
    y = w.data.y.copy()
    X = w.data.X.copy()
    rng = np.random.default_rng(17)
    idx = rng.choice(y.size, max(1, y.size * 3 // 100), replace=False)
    y[idx] = rng.choice(np.array([np.nan, np.inf, -np.inf], np.float32), idx.size)
    if matched:
        X[:, idx] = np.nan
    label = "generation P=3000 n=%d, 3%% invalid targets%s" % (
        n, ", NaN inputs there" if matched else "")
    _say(label)
    F = _run(gp, w.pop.nodes, w.pop.offsets, w.pop.consts, X, y, w.tax, w.allowed_mask)
    rep = _gate(F, w.pop.nodes, w.pop.offsets, w.pop.consts, X, y, w.tax,
                w.allowed_mask, label)
    assert not np.isnan(F).any()
    if matched:
        assert np.isfinite(F).sum() > 0 and np.isinf(F).sum() > 0
    else:
        assert np.all(np.isinf(F))


def test_matched_invalid_pairs_exact():
    """Hand-computed: outputs inf, NaN, -inf against NaN, inf, -inf targets
    are matched (no error); the finite cases give an exact MSE."""
    gp = _need_gpu()
    from oracle import EXP, LOAD, SIN
    inf, nan = np.inf, np.nan
    n = 300                       # a ragged sub-tile as well
    x = np.tile(np.array([inf, 0.5, -inf, 2.0, 89.0, 1.0], np.float32), n // 6)
    y = np.tile(np.array([nan, 1.5, -inf, 2.0, inf, 3.0], np.float32), n // 6)
    X = x.reshape(1, -1)
    progs = [[LOAD], [LOAD, EXP], [LOAD, SIN]]
    lens = np.array([len(q) for q in progs], np.int64)
    off = np.zeros(len(progs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([t for q in progs for t in q], np.uint32)
    _say("matched invalid pairs")
    F = _run(gp, nodes, off, np.zeros(0, np.float32), X, y, 0.0, oracle.MASK_BENCH)
    # x0: cases inf/nan, -inf/-inf matched; 0.5 vs 1.5 -> 1; 2 vs 2 -> 0;
    # 89 vs inf: finite vs invalid -> +inf
    assert F[0] == np.inf
    F64, _, st = oracle.fitness(nodes, off, np.zeros(0, np.float32), X, y, 0.0)
    assert (st == 0).all() and not np.isnan(F64).any()
    assert np.array_equal(np.isinf(F), np.isinf(F64))
    fin = np.isfinite(F64)
    assert np.allclose(F[fin], F64[fin], rtol=1e-6, atol=0)
    # a program whose only mismatch is removed: exact value by hand
    x2 = np.tile(np.array([inf, 0.5, -inf, 2.0, 1.0], np.float32), 60)
    y2 = np.tile(np.array([nan, 1.5, inf, 2.0, 3.0], np.float32), 60)
    F2 = _run(gp, np.array([LOAD], np.uint32), [0, 1], np.zeros(0, np.float32),
              x2.reshape(1, -1), y2, 0.0, oracle.MASK_BENCH)
    assert F2[0] == (1.0 + 4.0) / 5.0


def test_generation_full_size_sampled():
    """Full generation launch (100,000 programs x 4,096 cases) gated on a
    seeded sample of 400 programs, stratified by length."""
    gp = _need_gpu()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation")
    _say("generation full size")
    F = _run(gp, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
             w.allowed_mask)
    rng = np.random.default_rng(42)
    L = w.pop.lengths
    idx = np.concatenate([rng.choice(np.nonzero(L == l)[0], 7, replace=False)
                          for l in range(3, 65)])[:400]
    sub = w.pop.take(idx)
    _gate(F[idx], sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y, w.tax,
          w.allowed_mask, "generation full (sampled)")
    # every structurally valid program got a number or +inf, never NaN
    assert not np.isnan(F).any()


def _full_size_sampled(gp, name, per_len, cap, seed):
    """Workload ``name`` at full size in the launch configuration bench.py times,
    gated on a seeded sample stratified by program length."""
    from paper_2607_06731_amd import synth
    w = synth.make_workload(name)
    _say("%s full size: %d programs x %d cases" % (name, w.pop.n_programs, w.data.n_cases))
    F = _run(gp, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
             w.allowed_mask)
    rng = np.random.default_rng(seed)
    L = w.pop.lengths
    idx = []
    for l in np.unique(L):
        pool = np.nonzero(L == l)[0]
        idx.append(rng.choice(pool, min(per_len, pool.size), replace=False))
    idx = rng.permutation(np.concatenate(idx))[:cap]
    sub = w.pop.take(idx)
    _gate(F[idx], sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y, w.tax,
          w.allowed_mask, "%s full (sampled %d)" % (name, idx.size))
    assert not np.isnan(F).any()


def test_uneven_full_size_sampled():
    """1,000,000 programs (lengths 3..128) x 16,384 cases, 10 variables."""
    _full_size_sampled(_need_gpu(), "uneven", per_len=4, cap=400, seed=43)


def test_precision_full_size_sampled():
    """50,000 programs x 1,048,576 cases, |y| up to 1e4."""
    _full_size_sampled(_need_gpu(), "precision", per_len=1, cap=62, seed=44)


# ------------------------------------------------------------ pins on GPU
def test_brute_force_special_values():
    gp = _need_gpu()
    from tests.test_oracle_pins import SPECIAL, THETA, brute_force_programs
    seqs = brute_force_programs(5)
    st, _ = oracle.validate(np.array([t for s in seqs for t in s], np.uint32),
                            np.concatenate([[0], np.cumsum([len(s) for s in seqs])]),
                            1, 2, oracle.MASK_BENCH)
    valid = [s for s, c in zip(seqs, st) if c == 0]
    assert len(valid) == 13989
    lens = np.array([len(s) for s in valid], np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([t for s in valid for t in s], np.uint32)
    consts = np.array([-0.0011], np.float32)
    x0 = np.repeat(np.array(SPECIAL, np.float32), 5)
    x1 = np.tile(np.array([0.0, -THETA, 1.0, 44.0, -89.0], np.float32), len(SPECIAL))
    X = np.stack([x0, x1]).astype(np.float32)
    y = (0.5 * x0 - x1).astype(np.float32)
    _say("brute force 13989 programs")
    F = _run(gp, nodes, off, consts, X, y, 0.0, oracle.MASK_BENCH)
    _gate(F, nodes, off, consts, X, y, 0.0, oracle.MASK_BENCH, "brute force")
    # plus the same programs on moderate inputs, where nearly all are finite
    rng = np.random.default_rng(9)
    X2 = rng.uniform(-2, 2, (2, 700)).astype(np.float32)
    y2 = rng.uniform(-1, 1, 700).astype(np.float32)
    F2 = _run(gp, nodes, off, consts, X2, y2, 1e-3, oracle.MASK_BENCH)
    _gate(F2, nodes, off, consts, X2, y2, 1e-3, oracle.MASK_BENCH, "brute force moderate")


def test_exact_family_bitwise():
    gp = _need_gpu()
    from tests.test_oracle_pins import exact_family
    pop, X, y = exact_family(n_programs=2000, n_cases=1024, seed=8)
    F64, mse, st = oracle.fitness(pop.nodes, pop.offsets, pop.consts, X, y, 0.0)
    F32, _, _ = oracle.fitness(pop.nodes, pop.offsets, pop.consts, X, y, 0.0, mode=oracle.M32E)
    # keep programs whose fp32 evaluation is exact and whose sum of squares
    # stays below 2^24 * 4^e (scaled partial sums exact in fp32)
    keep = (F64 == F32) & np.isfinite(F64) & (F64 * 1024 < 2 ** 24)
    assert keep.sum() > 500
    _say("exact family")
    F = _run(gp, pop.nodes, pop.offsets, pop.consts, X, y, 0.0, oracle.MASK_BENCH)
    assert np.array_equal(F[keep], F64[keep])


def test_const_index_family_bitwise():
    gp = _need_gpu()
    P = 1_000_000
    nodes = (oracle.CONST | (np.arange(P, dtype=np.uint32) << 8)).astype(np.uint32)
    offsets = np.arange(P + 1, dtype=np.int64)
    consts = (np.arange(P) % 4096).astype(np.float32)
    X = np.zeros((1, 4), np.float32)
    y = np.zeros(4, np.float32)
    _say("const index family 1e6")
    F = _run(gp, nodes, offsets, consts, X, y, 0.0, oracle.MASK_BENCH)
    assert np.array_equal(F, (np.arange(P) % 4096).astype(np.float64) ** 2)


def test_quadratic_root_translation():
    gp = _need_gpu()
    from tests.test_oracle_pins import _quadratic_data, prog
    from oracle import ADD, DIV, MUL, SQRT, SUB
    X = _quadratic_data(4096, seed=3)
    a, b, c = (X[i].astype(np.float64) for i in range(3))
    root = (-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)
    p = prog(("x", 1), ("x", 1), MUL, ("c", 0), ("x", 0), MUL, ("x", 2), MUL, SUB,
             SQRT, ("x", 1), SUB, ("x", 0), DIV, ("c", 1), MUL)
    y = root.astype(np.float32)
    consts = np.array([4, 0.5], np.float32)
    _say("quadratic root")
    F = _run(gp, p, [0, p.size], consts, X, y, 0.0, oracle.MASK_BENCH)
    F64, _, _ = oracle.fitness(p, [0, p.size], consts, X, y, 0.0)
    assert abs(F[0] - F64[0]) <= 1e-4 * F64[0] + 1e-10


def test_precision_pin_million_cases():
    """c0 = 0 against y_i = 16((i mod 1024) - 511.5): exact MSE known."""
    gp = _need_gpu()
    from fractions import Fraction
    n, m, h = 1 << 20, 1024, 16.0
    i = np.arange(n)
    y = (h * ((i % m) - (m - 1) / 2.0)).astype(np.float32)
    X = np.zeros((1, n), np.float32)
    nodes = np.array([oracle.CONST], np.uint32)
    _say("precision pin 2^20 cases")
    F = _run(gp, nodes, [0, 1], np.array([0.0], np.float32), X, y, 0.0, oracle.MASK_BENCH)
    exact = float(Fraction(int(h) ** 2 * (m * m - 1), 12))
    assert abs(F[0] - exact) <= 1e-9 * exact


# ------------------------------------------------------------ edge cases
def test_invalid_programs_get_status_and_nan():
    gp = _need_gpu()
    from oracle import ADD, CONST, LOAD, SIN
    P = [
        [LOAD | (0 << 8), LOAD | (1 << 8), ADD],   # ok
        [],                                          # empty
        [LOAD | (0 << 8), 200],                      # bad op
        [LOAD | (7 << 8)],                           # bad var
        [CONST | (5 << 8)],                          # bad const
        [LOAD | (0 << 8), ADD],                      # underflow
        [LOAD] * 33 + [ADD] * 32,                    # too deep
        [LOAD, LOAD],                                # final depth 2
        [LOAD, SIN],                                 # disallowed below
    ]
    lens = np.array([len(p) for p in P], np.int64)
    off = np.zeros(len(P) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([t for p in P for t in p], np.uint32)
    consts = np.array([1.0], np.float32)
    X = np.ones((2, 100), np.float32)
    y = np.zeros(100, np.float32)
    mask = oracle.MASK_BENCH & ~(1 << SIN)
    _say("invalid programs")
    F, st = _run(gp, nodes, off, consts, X, y, 0.0, mask, status=True)
    st_o, _ = oracle.validate(nodes, off, 1, 2, mask)
    assert np.array_equal(st, st_o)
    assert F[0] == 4.0 and np.isnan(F[1:]).all()


def test_deep_and_long_programs():
    gp = _need_gpu()
    from oracle import ADD, COS, LOAD, MUL, SIN, SUB
    rng = np.random.default_rng(4)
    progs = []
    for d in (8, 9, 16, 17, 31, 32):     # class boundaries
        progs.append([LOAD | (int(rng.integers(0, 3)) << 8) for _ in range(d)] +
                     [int(rng.choice([ADD, SUB, MUL])) for _ in range(d - 1)])
    progs.append([LOAD] + [SIN, COS] * 2000)         # 4001 nodes
    lens = np.array([len(p) for p in progs], np.int64)
    off = np.zeros(len(progs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([t for p in progs for t in p], np.uint32)
    X = rng.uniform(-1, 1, (3, 3000)).astype(np.float32)
    y = rng.uniform(-1, 1, 3000).astype(np.float32)
    _say("deep and long programs")
    F = _run(gp, nodes, off, np.zeros(0, np.float32), X, y, 1e-3, oracle.MASK_BENCH)
    _gate(F, nodes, off, np.zeros(0, np.float32), X, y, 1e-3, oracle.MASK_BENCH, "deep/long")


def test_long_programs_staged_from_global_memory():
    """Programs of 150-260 nodes: a staging block's 128 programs span more
    nodes than its LDS node cache, so validation and staging read the nodes
    and constants from global memory (the short walks of a mask within the
    benchmark set, and the general walks of the full-table mask, which must
    give the same bits)."""
    gp = _need_gpu()
    from paper_2607_06731_amd import synth
    rng = np.random.default_rng(21)
    pop = synth.sample_programs(rng, rng.integers(150, 261, 1000), 4, synth.UNARY_2)
    assert (np.diff(pop.offsets)[:128].sum()) > 6656
    X = rng.uniform(-2, 2, (4, 1024)).astype(np.float32)
    y = rng.uniform(-2, 2, 1024).astype(np.float32)
    _say("long programs, uncached staging")
    F = _run(gp, pop.nodes, pop.offsets, pop.consts, X, y, 1e-3, oracle.MASK_BENCH)
    _gate(F, pop.nodes, pop.offsets, pop.consts, X, y, 1e-3, oracle.MASK_BENCH, "long/uncached")
    F_full = _run(gp, pop.nodes, pop.offsets, pop.consts, X, y, 1e-3, gp.GP_ALL_OPS)
    assert np.array_equal(F, F_full, equal_nan=True)


def test_no_variables_and_single_case():
    gp = _need_gpu()
    from oracle import ADD, CONST, MUL
    nodes = np.array([CONST | (0 << 8), CONST | (1 << 8), MUL, CONST | (2 << 8), ADD], np.uint32)
    consts = np.array([1.5, -2.0, 0.25], np.float32)
    X = np.zeros((0, 1), np.float32)
    y = np.array([1.0], np.float32)
    _say("no variables, one case")
    F = _run(gp, nodes, [0, 5], consts, X, y, 0.5, oracle.MASK_BENCH)
    assert F[0] == (-2.75 - 1.0) ** 2 + 0.5 * 5


def test_empty_population():
    gp = _need_gpu()
    _say("empty population")
    F = _run(gp, np.zeros(0, np.uint32), [0], np.zeros(0, np.float32),
             np.ones((1, 10), np.float32), np.zeros(10, np.float32), 0.0, 0)
    assert F.size == 0


def test_deterministic_and_batch_independent():
    gp = _need_gpu()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=6000, n_cases=4096)
    _say("determinism")
    F1 = _run(gp, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax, w.allowed_mask)
    F2 = _run(gp, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax, w.allowed_mask)
    assert np.array_equal(F1, F2)
    idx = np.random.default_rng(0).choice(6000, 500, replace=False)
    sub = w.pop.take(idx)
    F3 = _run(gp, sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y, w.tax, w.allowed_mask)
    assert np.array_equal(F3, F1[idx])


def test_commutativity_bitwise():
    gp = _need_gpu()
    from oracle import ADD, MUL
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=200, n_cases=2048)
    pop = w.pop
    progs = []
    for p in range(0, 100, 2):
        a = pop.nodes[pop.offsets[p]:pop.offsets[p + 1]]
        b = pop.nodes[pop.offsets[p + 1]:pop.offsets[p + 2]]
        for op in (ADD, MUL):
            progs.append(np.concatenate([a, b, [op]]))
            progs.append(np.concatenate([b, a, [op]]))
    lens = np.array([len(p) for p in progs], np.int64)
    off = np.zeros(len(progs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.concatenate(progs).astype(np.uint32)
    # both orders must land in the same stack-depth class (<= 8, 9..16,
    # 17..32): the class fixes the case tiling and hence the summation order
    _, md = oracle.validate(nodes, off, pop.consts.size, w.data.n_vars, w.allowed_mask)
    dclass = np.digitize(md, [8.5, 16.5])
    same = dclass[0::2] == dclass[1::2]
    assert same.sum() > 50
    _say("commutativity")
    F = _run(gp, nodes, off, pop.consts, w.data.X, w.data.y, w.tax, w.allowed_mask)
    assert np.array_equal(F[0::2][same], F[1::2][same])
