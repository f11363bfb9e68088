"""GPU parity of the integer point-to-point reward (the paper's Eq. 5,
StdFitFunc, and its Square, Cube and Hyper variants) through the C ABI
(gp_eval_reward) against the oracle.

Integer work decided by floating point: both sides take the per-case
decision in fp32 from the same fp32 output, so programs whose output is
exact in fp32 and fp64 alike (a variable, or a variable times a power of
two) must match the oracle bit for bit, over every branch of the reward
(zero pairs, sign flips, invalid pairs, rounding ties).  On the synthetic
workloads the program outputs themselves differ between an fp32 and an
fp64 evaluation; there the gate's reward mode applies: relative 1e-4 on
|F| + 0.01 M N, and a program outside that is certified only when its
total lies within the reward's bounds over the oracle's per-case output
windows (fp64, fp32 and perturbed-fp32 outputs, widened), else it fails.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import CONST, LOAD, MUL, gate

pytestmark = pytest.mark.gpu
M = 1e4
POWERS = (1, 2, 3, 8)


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


def _progs(progs):
    nodes = np.array([t for p in progs for t in p], np.uint32)
    off = np.concatenate([[0], np.cumsum([len(p) for p in progs])]).astype(np.int64)
    return nodes, off


def _special_cases(rng, n):
    """Outputs (rows 0..3) and targets covering every branch of the reward:
    zero pairs, one zero, sign flips, equal magnitudes, invalid values on
    either or both sides, exact rounding ties of M q for M = 8, and random
    ratios over many binades."""
    y = rng.normal(0, 1, n).astype(np.float32) * np.float32(10.0) ** rng.integers(-3, 4, n)
    ratio = rng.uniform(0, 1, n) ** rng.integers(1, 4, n)
    o = (y * ratio * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    swap = rng.random(n) < 0.5
    o[swap], y[swap] = y[swap].copy(), o[swap].copy()
    k = 0
    fixed = [(0.0, 0.0), (-0.0, 0.0), (0.0, 3.0), (-2.0, 0.0), (-2.0, 2.0), (2.0, -2.0),
             (5.0, 5.0), (np.inf, 1.0), (1.0, -np.inf), (np.nan, 1.0), (1.0, np.nan),
             (np.nan, np.nan), (np.inf, np.inf), (np.inf, np.nan), (-np.inf, 0.0),
             (1.0, 4.0), (3.0, 4.0), (4.0, 1.0), (-1.0, 4.0), (5.0, 10.0), (1.0, 8.0),
             (1e-38, 3e-38), (-1e-45, 1e-45), (3.4e38, -3.4e38), (1e-30, 1e30)]
    for a, b in fixed:
        o[k], y[k] = a, b
        k += 1
    # a block of ties for M = 8: q = k/16 (k odd) gives M q = k/2 exactly
    o[k:k + 8] = np.arange(1, 16, 2, dtype=np.float32)
    y[k:k + 8] = np.float32(16.0)
    return o, y


@pytest.mark.parametrize("power", POWERS)
@pytest.mark.parametrize("max_score", [8.0, M, 7.0, -3.0])
def test_reward_exact_on_exact_outputs(power, max_score):
    """Programs whose outputs are exact in any precision: bit-exact with the
    oracle's reward over every branch."""
    gp = _gp()
    rng = np.random.default_rng(100 + power)
    n = 3001                                   # several tiles and a ragged tail
    o, y = _special_cases(rng, n)
    X = np.stack([o, -o, o * np.float32(0.5), y]).astype(np.float32)
    consts = np.array([2.0, -0.25], np.float32)
    progs = [[LOAD | (0 << 8)], [LOAD | (1 << 8)], [LOAD | (2 << 8), CONST | (0 << 8), MUL],
             [LOAD | (0 << 8), CONST | (1 << 8), MUL], [LOAD | (3 << 8)]]
    nodes, off = _progs(progs)
    _say("reward exact outputs power=%d M=%g" % (power, max_score))
    R = gp.evaluate_reward(nodes, off, consts, X, y, max_score, power)
    ref, st = oracle.reward(nodes, off, consts, X, y, max_score, power)
    assert np.all(st == 0)
    assert np.array_equal(R, ref), (R, ref)
    # program 4 outputs y itself: every finite case scores M, every
    # invalid target is an invalid pair on both sides (+M)
    assert R[4] == max_score * n


def test_reward_ties_round_half_even():
    gp = _gp()
    o = np.arange(1, 16, 2, dtype=np.float32)
    y = np.full(8, 16.0, np.float32)
    nodes, off = _progs([[LOAD]])
    R = gp.evaluate_reward(nodes, off, np.zeros(1, np.float32), o[None, :], y, 8.0, 1)
    # 8 q = 0.5, 1.5, ..., 7.5: half to even gives 0, 2, 2, 4, 4, 6, 6, 8
    assert R[0] == 32.0


@pytest.mark.parametrize("power", POWERS)
@pytest.mark.parametrize("name,P,n", [("plain", None, None), ("generation", 4000, None),
                                      ("uneven", 3000, 4000), ("generation", 2000, 7)])
def test_reward_parity(name, P, n, power):
    gp = _gp()
    from paper_2607_06731_amd import synth
    w = synth.make_workload(name, n_programs=P, n_cases=n)
    label = "reward p=%d %s P=%d n=%d" % (power, name, w.pop.n_programs, w.data.n_cases)
    _say(label)
    R = gp.evaluate_reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, M,
                           power, w.allowed_mask)
    rep = gate.check(R, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, 0.0,
                     w.allowed_mask, max_score=M, reward_power=power)
    _say(label + ": " + rep.summary())
    assert rep.ok(), rep.failures[:10]
    ok = np.isfinite(R)
    assert np.all(R[ok] == np.round(R[ok]))
    assert np.all(np.abs(R[ok]) <= M * (1 + 1 / 11) * w.data.n_cases)


def test_reward_invalid_targets():
    gp = _gp()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=3000, n_cases=3000)
    y = w.data.y.copy()
    rng = np.random.default_rng(13)
    y[rng.choice(y.size, 60, replace=False)] = np.nan
    y[rng.choice(y.size, 30, replace=False)] = -np.inf
    _say("reward with invalid targets")
    R = gp.evaluate_reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, y, M, 2,
                           w.allowed_mask)
    rep = gate.check(R, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, y, 0.0,
                     w.allowed_mask, max_score=M, reward_power=2)
    _say("reward invalid targets: " + rep.summary())
    assert rep.ok(), rep.failures[:10]


def test_reward_population_independent_and_deterministic():
    gp = _gp()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=5000, n_cases=4096)
    R = gp.evaluate_reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, M, 8,
                           w.allowed_mask)
    idx = np.random.default_rng(4).choice(5000, 300, replace=False)
    sub = w.pop.take(idx)
    R_sub = gp.evaluate_reward(sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y, M, 8,
                               w.allowed_mask)
    _say("reward population independence")
    assert np.array_equal(R[idx], R_sub, equal_nan=True)
    R_again = gp.evaluate_reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X,
                                 w.data.y, M, 8, w.allowed_mask)
    assert np.array_equal(R, R_again, equal_nan=True)


def test_reward_full_size_sampled():
    """Full generation launch (100,000 programs x 4,096 cases) with the
    integer reward, gated on a seeded length-stratified sample."""
    gp = _gp()
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation")
    _say("reward generation full size")
    R = gp.evaluate_reward(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, M, 1,
                           w.allowed_mask)
    rng = np.random.default_rng(47)
    L = w.pop.lengths
    idx = np.concatenate([rng.choice(np.nonzero(L == l)[0], 6, replace=False)
                          for l in range(3, 65)])
    sub = w.pop.take(idx)
    rep = gate.check(R[idx], sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y, 0.0,
                     w.allowed_mask, max_score=M, reward_power=1)
    _say("reward generation full (sampled %d): %s" % (idx.size, rep.summary()))
    assert rep.ok(), rep.failures[:10]
    assert np.isfinite(R).all()
