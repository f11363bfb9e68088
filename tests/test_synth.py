"""The seeded workload generator produces valid programs with the stated
length laws (checked with the oracle's validator)."""
import numpy as np
import pytest

import oracle
from paper_2607_06731_amd import synth


@pytest.mark.parametrize("name,P", [("plain", 1000), ("generation", 5000), ("uneven", 20000),
                                    ("precision", 2000)])
def test_programs_valid_and_lengths(name, P):
    w = synth.make_workload(name, n_programs=P, n_cases=256)
    st, md = oracle.validate(w.pop.nodes, w.pop.offsets, w.pop.consts.size,
                             w.data.n_vars, w.allowed_mask)
    assert np.all(st == 0)
    assert md.max() <= 32
    L = w.pop.lengths
    lo, hi = {"plain": (3, 32), "generation": (3, 64), "uneven": (3, 128),
              "precision": (3, 64)}[name]
    assert L.min() >= lo and L.max() <= hi
    if name == "uneven":
        # clip(Geom(1/24), 3, 128): mean about 24, ~12% at the lower clip
        assert 22.5 < L.mean() < 25.5
        assert 0.10 < np.mean(L == 3) < 0.14


def test_deterministic():
    a = synth.make_workload("generation", n_programs=500, n_cases=64)
    b = synth.make_workload("generation", n_programs=500, n_cases=64)
    assert np.array_equal(a.pop.nodes, b.pop.nodes)
    assert np.array_equal(a.data.X, b.data.X) and np.array_equal(a.data.y, b.data.y)


def test_take_reindexes_constants():
    w = synth.make_workload("generation", n_programs=200, n_cases=64)
    idx = np.array([5, 17, 3, 199])
    sub = w.pop.take(idx)
    F_all, _, _ = oracle.fitness(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X,
                                 w.data.y, w.tax, w.allowed_mask)
    F_sub, _, _ = oracle.fitness(sub.nodes, sub.offsets, sub.consts, w.data.X,
                                 w.data.y, w.tax, w.allowed_mask)
    assert np.array_equal(F_all[idx], F_sub, equal_nan=True)


def test_workload_shapes():
    d = synth.make_dataset("precision", n_cases=4096)
    assert d.X.shape == (3, 4096) and d.X.dtype == np.float32
    assert np.abs(d.y).max() == pytest.approx(1e4, rel=1e-6)
    runs = synth.make_serving_runs(8)
    for r in runs:
        assert 1 <= r.data.n_vars <= 20 and 256 <= r.data.n_cases <= 65536


def test_gcl_sampler_valid_and_covers_the_command_table():
    w = synth.make_workload("gcl", n_programs=3000, n_cases=64)
    st, md = oracle.validate(w.pop.nodes, w.pop.offsets, w.pop.consts.size,
                             w.data.n_vars, w.allowed_mask)
    assert np.all(st == 0)
    assert md.max() <= 32
    L = w.pop.lengths
    assert L.min() >= 3 and L.max() <= 48
    ops = np.bincount(w.pop.nodes & 0xFF, minlength=synth.N_OPS)
    assert ops.size == synth.N_OPS and np.all(ops > 0)       # every command occurs
    # COPY/PASTE names stay below 16
    vp = (w.pop.nodes & 0xFF) >= synth.COPY
    assert np.all((w.pop.nodes[vp] >> 8) < synth.GCL_VARS)
