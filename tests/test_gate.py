"""The parity gate on the CPU: it passes the oracle's own values, catches a
planted error, and certifies fp32 effects only when the oracle's
fp32-emulating modes explain them (all three fitness functions); a
certified program's device value must still lie in the envelope of the
oracle's runs, and NaN is reserved for structurally invalid programs."""
import math

import numpy as np
import pytest

import oracle
from oracle import gate


def _workload():
    from paper_2607_06731_amd import synth
    return synth.make_workload("generation", n_programs=300, n_cases=512)


def test_mse_gate_passes_oracle_and_fails_planted_error():
    w = _workload()
    F64, _, st = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X,
                                w.data.y, w.tax, w.allowed_mask)
    rep = gate.check(F64, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                     w.tax, w.allowed_mask)
    assert rep.ok() and rep.n_pass == rep.n
    F32, _, _ = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X,
                               w.data.y, w.tax, w.allowed_mask, oracle.M32E)
    rep = gate.check(F32, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                     w.tax, w.allowed_mask)
    assert rep.ok()                       # fp32 rounding is certified, not failed
    bad = F64.copy()
    fin = np.nonzero(np.isfinite(bad))[0][:5]
    bad[fin] *= 1.001                     # a planted 0.1% error
    rep = gate.check(bad, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                     w.tax, w.allowed_mask)
    assert rep.n_fail >= 4


def test_correlation_gate_passes_oracle_and_fails_planted_error():
    w = _workload()
    S64, _, st = oracle.correlation(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X,
                                    w.data.y, 1e4, w.allowed_mask)
    args = (w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, 0.0,
            w.allowed_mask)
    rep = gate.check(S64, *args, max_score=1e4)
    assert rep.ok() and rep.n_pass == rep.n
    S32, _, _ = oracle.correlation(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X,
                                   w.data.y, 1e4, w.allowed_mask, oracle.M32E)
    assert gate.check(S32, *args, max_score=1e4).ok()
    bad = S64.copy()
    big = np.nonzero(np.abs(bad) > 1e3)[0][:5]
    assert big.size == 5
    bad[big] *= 1.001
    assert gate.check(bad, *args, max_score=1e4).n_fail >= 4


def test_reward_gate_passes_oracle_and_fails_planted_error():
    w = _workload()
    args = (w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, 0.0,
            w.allowed_mask)
    for power in (1, 8):
        R64, st = oracle.reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                                1e4, power, w.allowed_mask)
        rep = gate.check(R64, *args, max_score=1e4, reward_power=power)
        assert rep.ok() and rep.n_pass == rep.n
        R32, _ = oracle.reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                               1e4, power, w.allowed_mask, oracle.M32E)
        rep = gate.check(R32, *args, max_score=1e4, reward_power=power)
        assert rep.ok(), rep.failures
        # a planted error of 0.2 M per case on a few programs
        bad = R64.copy()
        idx = np.nonzero(st == 0)[0][:6]
        bad[idx] += 0.2e4 * w.data.n_cases
        rep = gate.check(bad, *args, max_score=1e4, reward_power=power)
        assert rep.n_fail >= 5, rep.summary()


def test_reward_window_brackets_oracle_modes():
    """The output window of every sampled program holds the oracle's own
    fp64 and fp32 totals, and is tight for most programs."""
    w = _workload()
    for power in (1, 3):
        R64, st = oracle.reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                                1e4, power, w.allowed_mask)
        R32, _ = oracle.reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                               1e4, power, w.allowed_mask, oracle.M32E_UP)
        widths = []
        for p in np.nonzero(st == 0)[0][:80]:
            prog = w.pop.nodes[w.pop.offsets[p]:w.pop.offsets[p + 1]]
            lo, hi = gate.reward_window(prog, w.pop.consts, w.data.X, w.data.y, 1e4, power,
                                        w.allowed_mask)
            assert lo <= R64[p] <= hi and lo <= R32[p] <= hi
            widths.append(hi - lo)
        assert np.median(widths) <= 1e-3 * 1e4 * w.data.n_cases


def _all_f32_between(a, b):
    """Every fp32 value in [a, b] (a <= b, finite, a small range)."""
    a32 = np.float32(a)
    if a32 < a:
        a32 = np.nextafter(a32, np.float32(np.inf))
    out = []
    x = a32
    while x <= b:
        out.append(x)
        x = np.nextafter(x, np.float32(np.inf))
    return np.array(out, np.float32)


def test_reward_window_bounds_against_brute_force():
    """window_bounds' least and greatest per-case reward equal those found
    by enumerating every fp32 value of the window (small windows around
    zero, around +-|y|, and away from both)."""
    rng = np.random.default_rng(31)
    tiny = float(np.finfo(np.float32).smallest_subnormal)
    cases = []
    for _ in range(40):
        y = np.float32(rng.choice([-1.0, 1.0]) * 10.0 ** rng.uniform(-3, 3))
        kind = rng.integers(0, 4)
        if kind == 0:
            c = float(y)                                   # around o = y
        elif kind == 1:
            c = -float(y)                                  # around o = -y
        elif kind == 2:
            c = 0.0                                        # around zero (subnormals)
        else:
            c = float(y) * rng.uniform(-3, 3)
        span = rng.integers(1, 300)
        step = tiny if kind == 2 else float(np.spacing(np.float32(abs(c) + 1e-30)))
        O = np.array([[c - span * step], [c + span * step * rng.uniform(0.2, 1.0)]])
        cases.append((O, y))
    cases.append((np.array([[np.nan], [1.0]]), np.float32(1.5)))     # a candidate invalid
    cases.append((np.array([[np.inf], [np.nan]]), np.float32(2.0)))  # all invalid
    cases.append((np.array([[0.5], [0.5]]), np.float32(np.nan)))     # invalid target
    for M in (1e4, 8.0, -3.0):
        for power in (1, 2, 3, 8):
            for O, y in cases:
                rmin, rmax, a, b = gate.window_bounds(O, np.array([y]), M, power)
                fin = np.isfinite(O[:, 0])
                vals = []
                if fin.any():
                    xs = _all_f32_between(a[0], b[0]).astype(np.float64)
                    vals.append(oracle.case_rewards(xs, np.full(xs.size, y), M, power))
                if not fin.all():
                    vals.append(oracle.case_rewards(np.array([np.nan]), np.array([y]), M,
                                                    power))
                v = np.concatenate(vals)
                assert rmin[0] == v.min() and rmax[0] == v.max(), (O, y, M, power)


def _one(toks, consts=()):
    out = []
    for t in toks:
        if isinstance(t, tuple):
            out.append((oracle.LOAD if t[0] == "x" else oracle.CONST) | (t[1] << 8))
        else:
            out.append(t)
    nodes = np.array(out, np.uint32)
    return nodes, np.array([0, nodes.size], np.int64), np.array(consts, np.float32)


def _chaotic_case():
    """sin(exp(6 x0)) on x0 in (-3, 3): exp reaches ~6.6e7, where one fp32
    ulp of its result moves the sine anywhere in [-1, 1]."""
    rng = np.random.default_rng(5)
    X = rng.uniform(-3, 3, (1, 512)).astype(np.float32)
    y = rng.uniform(-1, 1, 512).astype(np.float32)
    nodes, offs, consts = _one([("x", 0), ("c", 0), oracle.MUL, oracle.EXP, oracle.SIN], [6.0])
    return nodes, offs, consts, X, y


def test_chaotic_excuse_is_bounded_by_the_envelope():
    nodes, offs, consts, X, y = _chaotic_case()
    args = (nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH)
    runs = [oracle.fitness(nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH, m)[0][0]
            for m in [oracle.M64, oracle.M32E, oracle.M32E_UP, oracle.M32E_DN] +
            [oracle.M32E_RAND + s for s in range(gate.N_RANDOM)]]
    lo, hi = min(runs), max(runs)
    assert hi - lo > 1e-3 * hi                       # the program is chaotic
    # a value among the runs is certified as chaotic ...
    rep = gate.check(np.array([runs[2]]), *args)
    assert rep.ok() and (rep.n_chaotic == 1 or rep.n_pass == 1), rep.summary()
    # ... one far outside their envelope is not, however chaotic the program
    for planted in (hi + 5 * (hi - lo) + 1.0, max(lo - 5 * (hi - lo) - 1.0, -1.0)):
        rep = gate.check(np.array([planted]), *args)
        assert rep.n_fail == 1, (planted, rep.summary())


def test_certified_class_flip_bounds_a_finite_device_value():
    """x0 * 1e19 squared: in fp32 the MSE is near FLT_MAX; a device class
    flip to a finite value is certified only inside the runs' envelope."""
    X = np.array([[1.0, 1.0, 1.0, 1.0]], np.float32)
    y = np.zeros(4, np.float32)
    c = float(np.float32(1.8446742e19))            # c^2 ~ FLT_MAX: at the class edge
    nodes, offs, consts = _one([("x", 0), ("c", 0), oracle.MUL], [c])
    args = (nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH)
    F64 = oracle.fitness(nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH)[0][0]
    assert math.isfinite(F64)
    # the oracle's own value passes, a planted infinite class fails
    assert gate.check(np.array([F64]), *args).n_pass == 1
    assert gate.check(np.array([math.inf]), *args).n_fail == 1
    assert gate.check(np.array([F64 * 0.5]), *args).n_fail == 1


def test_nan_is_reserved_for_invalid_programs():
    w = _workload()
    F64, _, st = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X,
                                w.data.y, w.tax, w.allowed_mask)
    fin = np.nonzero(np.isfinite(F64) & (st == 0))[0][:3]
    inf = np.nonzero(np.isinf(F64) & (st == 0))[0][:3]
    assert fin.size == 3 and inf.size == 3
    bad = F64.copy()
    bad[fin] = np.nan
    bad[inf] = np.nan
    rep = gate.check(bad, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                     w.tax, w.allowed_mask)
    assert rep.n_fail == 6
    assert sum(1 for f in rep.failures if f[1] == "valid program NaN") == 6


def test_mse_gate_with_invalid_targets():
    """3% NaN/+-inf targets: the oracle's own values pass (finite and +inf
    classes both occur), the fp32 evaluation is certified, a swapped class
    fails."""
    w = _workload()
    y = w.data.y.copy()
    rng = np.random.default_rng(9)
    idx = rng.choice(y.size, y.size * 3 // 100, replace=False)
    y[idx] = rng.choice(np.array([np.nan, np.inf, -np.inf], np.float32), idx.size)
    args = (w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, y, w.tax, w.allowed_mask)
    F64, _, st = oracle.fitness(*args)
    assert not np.any(np.isnan(F64[st == 0]))
    rep = gate.check(F64, *args)
    assert rep.ok() and rep.n_pass == rep.n
    F32, _, _ = oracle.fitness(*args, mode=oracle.M32E)
    assert gate.check(F32, *args).ok()


def test_correlation_floor_only_near_zero():
    """A planted error of 1e-3 relative on a well-conditioned program with a
    small but clearly nonzero r^4 fails: the absolute floor (1e-9 M N) no
    longer hides it."""
    rng = np.random.default_rng(2)
    n = 4096
    X = rng.uniform(-1, 1, (2, n)).astype(np.float32)
    M = 1e4
    hit = None
    for a in np.linspace(0.005, 0.05, 40):
        y = (X[1] + np.float32(a) * X[0]).astype(np.float32)
        nodes, offs, consts = _one([("x", 0), ("c", 0), oracle.MUL], [1.5])
        S, r, st = oracle.correlation(nodes, offs, consts, X, y, M, oracle.MASK_BENCH)
        if 2e-7 < r[0] ** 4 < 2e-6:
            hit = (y, nodes, offs, consts, S[0], r[0])
            break
    assert hit is not None
    y, nodes, offs, consts, S, r = hit
    args = (nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH)
    assert gate.check(np.array([S]), *args, max_score=M).n_pass == 1
    planted = S * (1 + 1e-3)
    assert abs(planted - S) < 1e-9 * M * n       # inside the old floor
    assert gate.check(np.array([planted]), *args, max_score=M).n_fail == 1


def _window_bound_mse(f, lo, hi, fin, y):
    yy = y.astype(np.float64)
    v = fin & np.isfinite(yy)
    reach = np.where(v, np.maximum(hi - f, f - lo), 0.0)
    return float(np.sum(2 * np.abs(np.where(v, f - yy, 0.0)) * reach + reach ** 2)) / y.size


def test_mse_window_bound_holds_for_outputs_in_the_windows():
    """The MSE window bound is exact: outputs drawn anywhere in the per-case
    windows give an MSE within it; a device value beyond it (and outside
    the runs' envelope) fails, one inside it is excused."""
    nodes, offs, consts, X, y = _chaotic_case()
    f, lo, hi, fin = gate.output_windows(nodes, consts, X, y, oracle.MASK_BENCH)
    assert fin.all()
    bound = _window_bound_mse(f, lo, hi, fin, y)
    F64 = float(np.mean((f - y) ** 2))
    rng = np.random.default_rng(3)
    for _ in range(50):
        t = rng.uniform(0, 1, y.size)
        o = lo + t * (hi - lo)
        assert abs(float(np.mean((o - y) ** 2)) - F64) <= bound
    args = (nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH)
    assert gate.window_excuse(F64 + 0.9 * bound, F64, F64, nodes, consts, X, y,
                              oracle.MASK_BENCH)
    assert not gate.window_excuse(F64 + 1.1 * bound + 1e-4 * F64, F64, F64, nodes, consts, X,
                                  y, oracle.MASK_BENCH)
    runs = [oracle.fitness(nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH, m)[0][0]
            for m in [oracle.M64, oracle.M32E, oracle.M32E_UP, oracle.M32E_DN] +
            [oracle.M32E_RAND + s for s in range(gate.N_RANDOM)]]
    env = gate.envelope(runs)
    planted = max(env[1], F64 + bound) * 1.01 + 1e-3
    assert gate.check(np.array([planted]), *args).n_fail == 1


def test_correlation_window_bound_covers_outputs_in_the_windows():
    """A weakly correlated program whose outputs carry fp32 error: r over
    outputs drawn anywhere in the windows stays within the first-order
    bound (with its factor 2); a device value beyond the bound fails, one
    inside it is excused, and a correlation term below zero (an r^4 that
    no outputs can give) fails."""
    rng = np.random.default_rng(11)
    n = 2048
    X = rng.uniform(-3, 3, (2, n)).astype(np.float32)
    y = (X[1] + np.float32(0.02) * np.sin(X[0] * 40.0)).astype(np.float32)
    # exp(x0 * 6) / 7 + x1 * 1e-3: large, fp32-rounded outputs, weak r with y
    nodes, offs, consts = _one([("x", 0), ("c", 0), oracle.MUL, oracle.EXP, ("c", 1), oracle.DIV,
                                ("x", 1), ("c", 2), oracle.MUL, oracle.ADD], [6.0, 7.0, 1e-3])
    M = 1e4
    S, r, st, c1, c2 = oracle.correlation(nodes, offs, consts, X, y, M, oracle.MASK_BENCH,
                                          return_counts=True)
    f, lo, hi, fin = gate.output_windows(nodes, consts, X, y, oracle.MASK_BENCH)
    assert fin.all()
    yy = y.astype(np.float64)
    df, dy = f - f.mean(), yy - yy.mean()
    sxx, syy = df @ df, dy @ dy
    r0 = (df @ dy) / np.sqrt(sxx * syy)
    assert abs(r0 - r[0]) < 1e-9
    reach = np.maximum(hi - f, f - lo)
    dr = 2 * np.sum(np.abs(dy / np.sqrt(sxx * syy) - r0 * df / sxx) * reach)
    for _ in range(50):
        o = lo + rng.uniform(0, 1, n) * (hi - lo)
        do = o - o.mean()
        ro = (do @ dy) / np.sqrt((do @ do) * syy)
        assert abs(ro - r0) <= dr
    bound = M * n * (min(1.0, abs(r0) + dr) ** 4 - r0 ** 4)
    T = M * r0 ** 4 * n
    assert bound < 0.5 * T                       # the bound is informative here
    F = float(S[0])
    assert gate.window_excuse(F + 0.9 * bound, F, T, nodes, consts, X, y, oracle.MASK_BENCH, M)
    assert not gate.window_excuse(F + 1.1 * bound + 1e-4 * T, F, T, nodes, consts, X, y,
                                  oracle.MASK_BENCH, M)
    assert not gate.window_excuse(-1.0, F, T, nodes, consts, X, y, oracle.MASK_BENCH, M)
    args = (nodes, offs, consts, X, y, 0.0, oracle.MASK_BENCH)
    assert gate.check(np.array([F + 3 * bound + 1e-3 * T]), *args, max_score=M).n_fail == 1
