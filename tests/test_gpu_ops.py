"""Per-case checks through gp_predict (the ExecuteGenome-style utility).

Each op is run as a one-op program over dense sweeps of inputs and compared,
case by case, with the oracle's M32E mode (the correctly rounded fp32 value
of the fp64 result).  Bounds: +, -, *, |.| and protected DIV exact (they
are correctly rounded in fp32), elementary functions
and the square root within 2 ulps (the envelope the parity gate's chaos
certificate assumes).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import (ABS, ADD, CONST, COS, DIV, EXP, LOAD, LOG, MUL, SIN, SQRT,
                    SUB)

pytestmark = pytest.mark.gpu

ULP_BOUND = {SIN: 2.0, COS: 2.0, EXP: 2.0, LOG: 2.0, SQRT: 2.0, ABS: 0.0,
             ADD: 0.0, SUB: 0.0, MUL: 0.0, DIV: 0.0}


def _gp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_06731_amd as gp
    gp.lib()
    return gp


def _say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def ulp_err(got, ref):
    """|got - ref| in units of the fp32 spacing at ref (both fp32 values)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    both_nan = np.isnan(got) & np.isnan(ref)
    same_inf = np.isinf(got) & np.isinf(ref) & (np.sign(got) == np.sign(ref))
    sp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    e = np.abs(got - ref) / sp
    e[both_nan | same_inf | (got == ref)] = 0.0
    e[np.isnan(got) != np.isnan(ref)] = np.inf
    return e


def sweep(rng, n=200_000):
    parts = [rng.uniform(-4, 4, n), rng.uniform(-100, 100, n),
             rng.uniform(-1e4, 1e4, n), rng.uniform(-2e5, 2e5, n // 4),
             np.exp(rng.uniform(-80, 80, n)) * rng.choice([-1, 1], n),
             np.array([0.0, -0.0, 1e-40, -1e-40, np.inf, -np.inf, np.nan,
                       1e38, -1e38, 88.0, 88.7, 89.0, 0.001, -0.001,
                       float(np.float32(0.001)), float(np.nextafter(np.float32(0.001), 1)),
                       131072.0, 131072.5, -131072.0, 3e6])]
    k = np.arange(-40000, 40000)
    parts.append(k * np.pi)
    parts.append((k + 0.5) * np.pi)
    x = np.concatenate(parts).astype(np.float32)
    return np.concatenate([x, np.nextafter(x, np.float32(np.inf))])


@pytest.mark.parametrize("op", [SIN, COS, EXP, LOG, SQRT, ABS])
def test_unary_ulps(op):
    gp = _gp()
    x = sweep(np.random.default_rng(op))
    X = x.reshape(1, -1)
    prog = np.array([LOAD, op], np.uint32)
    _say("unary op %d on %d inputs" % (op, x.size))
    got = gp.predict(prog, [0, 2], np.zeros(0, np.float32), X)[0]
    ref = oracle.program_outputs(prog, [], X, mode=oracle.M32E)
    e = ulp_err(got, ref)
    worst = np.argsort(e)[-5:]
    _say("op %d: max ulp %.3f mean %.4f worst x=%s" % (op, e.max(), e.mean(), x[worst]))
    assert e.max() <= ULP_BOUND[op], (x[worst], got[worst], ref[worst])


@pytest.mark.parametrize("op", [ADD, SUB, MUL, DIV])
def test_binary_ulps(op):
    gp = _gp()
    rng = np.random.default_rng(10 + op)
    a = sweep(rng, 50_000)
    b = rng.permutation(sweep(rng, 50_000))
    n = min(a.size, b.size)
    X = np.stack([a[:n], b[:n]])
    for prog in ([LOAD, LOAD | (1 << 8), op], [LOAD | (1 << 8), LOAD, op]):
        prog = np.array(prog, np.uint32)
        got = gp.predict(prog, [0, 3], np.zeros(0, np.float32), X)[0]
        ref = oracle.program_outputs(prog, [], X, mode=oracle.M32E)
        e = ulp_err(got, ref)
        _say("op %d: max ulp %.3f" % (op, e.max()))
        assert e.max() <= ULP_BOUND[op]


def test_leaf_folding_forms():
    """Every staged form: plain leaves, top OP leaf (variable and constant),
    f(leaf) (variable and constant), stack binary ops, against M32E
    per case (exact ops only, so the comparison is bitwise)."""
    gp = _gp()
    c = lambda j: CONST | (j << 8)
    v = lambda j: LOAD | (j << 8)
    progs = [
        [v(0)], [c(0)],
        [v(0), v(1), ADD], [v(0), c(1), SUB], [c(0), v(1), MUL], [c(0), c(1), DIV],
        [v(0), ABS], [c(1), ABS], [v(1), v(0), ABS, SUB],
        [v(0), v(1), v(0), MUL, SUB, c(1), DIV, ABS],
        [v(0), v(1), ADD, v(0), v(1), SUB, MUL],
        [c(0), v(0), v(1), v(0), v(1), ADD, SUB, MUL, DIV],
    ]
    lens = np.array([len(p) for p in progs], np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([t for p in progs for t in p], np.uint32)
    consts = np.array([1.25, -3.5], np.float32)
    rng = np.random.default_rng(2)
    X = rng.uniform(-5, 5, (2, 3000)).astype(np.float32)
    _say("leaf folding forms")
    got = gp.predict(nodes, off, consts, X)
    for p in range(len(progs)):
        ref = oracle.program_outputs(nodes[off[p]:off[p + 1]], consts, X, mode=oracle.M32E)
        assert np.array_equal(got[p].astype(np.float64), ref), p


def test_predict_invalid_rows_and_status():
    gp = _gp()
    import torch
    progs = [[LOAD, LOAD | (1 << 8), ADD], [LOAD, ADD], [LOAD | (5 << 8)], [LOAD, SIN]]
    lens = np.array([len(p) for p in progs], np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([t for p in progs for t in p], np.uint32)
    X = np.ones((2, 777), np.float32)
    pop = gp.DevicePopulation(nodes, off, np.zeros(0, np.float32))
    Xd = torch.from_numpy(X).cuda()
    out = torch.zeros((4, 800), dtype=torch.float32, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    _say("predict invalid rows")
    gp.gp_predict(pop.nodes, pop.offsets, pop.consts, Xd, out, st,
                  allowed_op_mask=oracle.MASK_BENCH & ~(1 << SIN))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(o[0, :777] == 2.0) and np.all(o[0, 777:] == 0.0)   # ld_out padding untouched
    assert np.isnan(o[1:, :777]).all()
    assert st.cpu().numpy().tolist() == [0, 5, 3, 2]


def test_predict_agrees_with_eval():
    """MSE recomputed from gp_predict outputs equals gp_eval's fitness
    within the compensated-sum error."""
    gp = _gp()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=300, n_cases=2000)
    _say("predict vs eval")
    f = gp.predict(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X).astype(np.float64)
    F = gp.evaluate(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
                    w.allowed_mask)
    fin = np.isfinite(f).all(axis=1)
    mse = ((f - w.data.y.astype(np.float64)) ** 2).mean(axis=1)
    Fp = np.where(fin & (mse <= np.finfo(np.float32).max), mse + w.tax * w.pop.lengths, np.inf)
    both = np.isfinite(Fp)
    assert np.array_equal(both, np.isfinite(F))
    assert np.all(np.abs(F[both] - Fp[both]) <= 1e-6 * np.abs(Fp[both]) + 1e-12)


def test_overlapping_node_ranges():
    """Programs may share nodes through their offsets; each staged program
    gets its own range.  If the staged programs together would need more
    than n_nodes entries, no program of the call is evaluated and all get
    GP_PROG_BAD_OFFSETS (never a write outside the staging buffer)."""
    gp = _gp()
    v = lambda j: LOAD | (j << 8)
    nodes = np.array([v(0), v(1), ADD, v(0), MUL], np.uint32)
    rng = np.random.default_rng(4)
    X = rng.uniform(-2, 2, (2, 700)).astype(np.float32)
    y = rng.uniform(-2, 2, 700).astype(np.float32)
    consts = np.zeros(0, np.float32)
    _say("overlapping node ranges")
    # p0 = nodes[0:3], p1 = nodes[3:0] (decreasing), p2 = nodes[0:5]: 5 staged entries fit
    off = np.array([0, 3, 0, 5], np.int64)
    F, st = gp.evaluate(nodes, off, consts, X, y, 0.0, 0, return_status=True)
    assert st.tolist() == [0, 8, 0] and np.isnan(F[1])
    for p in (0, 2):
        sn, so = oracle.subset(nodes, off, [p])
        ref, _, _ = oracle.fitness(sn, so, consts, X, y)
        assert abs(F[p] - ref[0]) <= 1e-4 * abs(ref[0]) + 1e-12
    # p0 = p2 = nodes[0:5]: 6 staged entries > 5 nodes
    off = np.array([0, 5, 0, 5], np.int64)
    F, st = gp.evaluate(nodes, off, consts, X, y, 0.0, 0, return_status=True)
    assert st.tolist() == [8, 8, 8] and np.isnan(F).all()


def test_packed_restaging_gives_the_same_bits():
    """A decreasing offset pair anywhere in a call (after which node ranges
    may overlap) makes every program be staged again, packed, instead of
    in place by the validating walk: on the generation workload's programs
    the scores are bit-identical either way, and the extra program gets
    GP_PROG_BAD_OFFSETS."""
    gp = _gp()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=20_000, n_cases=2_000)
    _say("staging in place and packed, P=20000 n=2000")
    F0, st0 = gp.evaluate(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
                          w.allowed_mask, return_status=True)
    off = np.concatenate([w.pop.offsets, [w.pop.offsets[-1] - 7]])
    F1, st1 = gp.evaluate(w.pop.nodes, off, w.pop.consts, w.data.X, w.data.y, w.tax,
                          w.allowed_mask, return_status=True)
    assert st1[-1] == 8 and np.isnan(F1[-1])
    assert np.array_equal(st0, st1[:-1])
    assert (st0 == 0).sum() > 19_000
    assert np.array_equal(F0.view(np.uint64), F1[:-1].view(np.uint64))


def test_constant_subtrees_fold_to_the_same_bits():
    """Constant subtrees are computed once while staging, with the
    interpreter's own arithmetic: every per-case output must equal, bit for
    bit, the same program with each constant read from an input row that
    holds that constant in every case (which the interpreter evaluates per
    case)."""
    gp = _gp()
    c = lambda j: CONST | (j << 8)
    v = lambda j: LOAD | (j << 8)
    consts = np.array([0.75, -2.5, 1e-4, 3e5, 88.5, -0.0, 1e30], np.float32)
    n_c = consts.size
    shapes = [
        [c(0), SIN], [c(3), COS, c(1), MUL], [c(4), EXP, c(6), MUL], [c(2), LOG],
        [c(1), SQRT, c(0), DIV], [c(5), ABS, c(1), ADD], [c(0), c(1), DIV, SIN, v(0), ADD],
        [v(0), c(0), c(1), MUL, SUB], [c(0), v(0), c(1), MUL, ADD],
        [c(1), c(2), DIV, v(0), MUL, c(3), SIN, c(4), COS, MUL, SUB],
        [c(6), c(6), MUL, v(0), ADD],                    # overflow in the folded part
        [v(0), c(2), c(5), SUB, DIV],                    # protected division by a small constant
        [c(0), EXP, EXP, EXP, LOG, c(1), COS, ADD],
        # runs of constants longer than staging holds back (16): the
        # excess is pushed as runtime values and still computes the same
        [c(j % 5) for j in range(20)] + [ADD, SUB] * 9 + [MUL, v(0), ADD],
        [c(j % 3) for j in range(24)] + [SIN] + [ADD] * 23 + [v(0), MUL],
        [c(0)] * 17 + [v(0)] + [c(1)] * 14 + [SUB] * 31 + [COS],
        [v(0)] + [c(j % 4) for j in range(31)] + [DIV, ADD] * 15 + [ADD],
    ]
    # the same programs with constant j read from input row 1 + j
    as_vars = [[v(1 + (t >> 8)) if (t & 0xFF) == CONST else t for t in prog] for prog in shapes]
    rng = np.random.default_rng(9)
    X = np.empty((1 + n_c, 3000), np.float32)
    X[0] = rng.uniform(-4, 4, 3000)
    X[1:] = consts[:, None]
    for group in (shapes, as_vars):
        lens = [len(p) for p in group]
        assert max(lens) <= 64
    flat = lambda g: (np.array([t for p in g for t in p], np.uint32),
                      np.concatenate([[0], np.cumsum([len(p) for p in g])]).astype(np.int64))
    n1, o1 = flat(shapes)
    n2, o2 = flat(as_vars)
    _say("constant folding bit identity")
    got = gp.predict(n1, o1, consts, X)
    ref = gp.predict(n2, o2, consts, X)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), \
        np.nonzero(got.view(np.uint32) != ref.view(np.uint32))
