"""The parity gate on the CPU: it passes the oracle's own values, catches a
planted error, and certifies fp32 effects only when the oracle's
fp32-emulating modes explain them (both fitness functions)."""
import numpy as np

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
