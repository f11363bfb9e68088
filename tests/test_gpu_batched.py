"""gp_eval_batched: many requests, each with its own program arrays and its
own dataset, in one launch.  Each program's fitness must be bit-identical to
scoring its request alone with gp_eval (batch-composition independence of
the serving path), and the batched results pass the oracle's parity gate."""
import sys

import numpy as np
import pytest

import oracle
from oracle import gate

pytestmark = pytest.mark.gpu


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


def _requests(n_req=12, seed=5, max_pop=3000, max_cases=20000):
    from paper_2607_06731_amd import synth
    rng = np.random.default_rng(seed)
    runs = synth.make_serving_runs(6, seed=seed, max_cases=max_cases)
    reqs = []
    for _ in range(n_req):
        i = int(rng.integers(0, len(runs)))
        pop = synth.make_serving_request(rng, runs[i], min_pop=50, max_pop=max_pop)
        reqs.append((i, pop))
    return runs, reqs


def _run_batched(gp, runs, reqs, tax, extra_empty=()):
    """Upload, build the tables, launch once; returns per-request (F, status)."""
    import torch
    data = [gp.DeviceDataset(r.data.X, r.data.y) for r in runs]
    dsets = gp.table_tensor([gp.dataset_entry(d, tax) for d in data])
    entries, keep, outs = [], [], []
    for k, (i, pop) in enumerate(reqs):
        dp = gp.DevicePopulation(pop.nodes, pop.offsets, pop.consts)
        out = torch.full((dp.n_programs,), -1.0, dtype=torch.float64, device="cuda")
        st = torch.full((dp.n_programs,), -1, dtype=torch.int32, device="cuda")
        entries.append(gp.request_entry(dp, i, out, st))
        keep.append(dp)
        outs.append((out, st))
        if k in extra_empty:
            empty = gp.DevicePopulation(np.zeros(0, np.uint32), np.zeros(1, np.int64),
                                        np.zeros(0, np.float32))
            e_out = torch.empty(0, dtype=torch.float64, device="cuda")
            entries.append(gp.request_entry(empty, 0, e_out))
            keep.append((empty, e_out))
    reqs_t = gp.table_tensor(entries)
    total_p = sum(e.n_programs for e in entries)
    total_n = sum(e.n_nodes for e in entries)
    gp.gp_eval_batched(reqs_t, dsets, total_p, total_n, max(d.n_vars for d in data),
                       max(d.n_cases for d in data))
    torch.cuda.synchronize()
    return [(o.cpu().numpy(), s.cpu().numpy()) for o, s in outs]


def test_batched_equals_alone():
    gp = _gp()
    runs, reqs = _requests()
    tax = 1e-3
    _say("batched %d requests, %d programs" % (len(reqs), sum(p.n_programs for _, p in reqs)))
    got = _run_batched(gp, runs, reqs, tax, extra_empty=(0, 5))
    for (i, pop), (F, st) in zip(reqs, got):
        run = runs[i]
        alone = gp.evaluate(pop.nodes, pop.offsets, pop.consts, run.data.X, run.data.y, tax, 0)
        assert (st == 0).all()
        assert np.array_equal(F, alone, equal_nan=True)


def test_batched_parity_gate():
    """Batched results against the fp64 oracle (smaller requests)."""
    gp = _gp()
    runs, reqs = _requests(n_req=5, seed=21, max_pop=400, max_cases=3000)
    tax = 1e-3
    _say("batched parity, %d requests" % len(reqs))
    got = _run_batched(gp, runs, reqs, tax)
    for (i, pop), (F, st) in zip(reqs, got):
        run = runs[i]
        rep = gate.check(F, pop.nodes, pop.offsets, pop.consts, run.data.X, run.data.y, tax,
                         oracle.MASK_BENCH)
        _say(rep.summary())
        assert rep.ok(), rep.failures


def test_batched_mixed_invalid_programs():
    """Invalid programs inside a request get NaN and their status; the
    request's other programs are unaffected."""
    gp = _gp()
    runs, reqs = _requests(n_req=3, seed=33, max_pop=300, max_cases=2000)
    i, pop = reqs[1]
    nodes = pop.nodes.copy()
    bad_prog = [0, 7]
    nodes[pop.offsets[0]] = oracle.LOAD | (200 << 8)            # variable out of range
    nodes[pop.offsets[7]] = 99                                  # unknown op
    from paper_2607_06731_amd.synth import Population
    reqs[1] = (i, Population(nodes, pop.offsets, pop.consts))
    got = _run_batched(gp, runs, reqs, 0.0)
    F, st = got[1]
    assert st[0] == oracle.ST_BAD_VAR and st[7] == oracle.ST_BAD_OP
    assert np.isnan(F[bad_prog]).all()
    ok = np.setdiff1d(np.arange(F.size), bad_prog)
    run = runs[i]
    alone = gp.evaluate(nodes, pop.offsets, pop.consts, run.data.X, run.data.y, 0.0, 0)
    assert np.array_equal(F[ok], alone[ok], equal_nan=True)


def test_batched_rejects_bad_table():
    gp = _gp()
    import torch
    runs, reqs = _requests(2, seed=9, max_pop=500)
    i, pop0 = reqs[0]
    d = gp.DeviceDataset(runs[i].data.X, runs[i].data.y)
    pop = gp.DevicePopulation(pop0.nodes, pop0.offsets, pop0.consts)
    P = pop.n_programs
    dsets = gp.table_tensor([gp.dataset_entry(d, 0.0)])
    out = torch.empty(P, dtype=torch.float64, device="cuda")
    st = torch.empty(P, dtype=torch.int32, device="cuda")
    good = gp.request_entry(pop, 0, out, st)
    bad_ds = gp.request_entry(pop, 3, out, st)              # dataset out of range
    cases = [([bad_ds], P, pop.nodes.numel()),
             ([good], P + 1, pop.nodes.numel()),             # totals disagree with the table
             ([good], P, pop.nodes.numel() + 5)]
    for entries, tp, tn in cases:
        _say("bad table total_programs=%d total_nodes=%d" % (tp, tn))
        out.fill_(0.0)
        st.fill_(0)
        gp.gp_eval_batched(gp.table_tensor(entries), dsets, tp, tn, d.n_vars, d.n_cases)
        torch.cuda.synchronize()
        assert np.isnan(out.cpu().numpy()).all()
        assert (st.cpu().numpy() == 9).all()
    # host-side argument errors
    with pytest.raises(gp.GPError):
        gp.gp_eval_batched(gp.table_tensor([good]), gp.table_tensor([]), P, pop.nodes.numel(),
                           d.n_vars, d.n_cases)


def test_batched_tile_counts_of_mixed_sizes():
    """A smaller dataset can need more case tiles than the largest one of
    the call (33 sub-tiles make 17 tiles, 32 make 32): partial rows must be
    sized for both, and results stay equal to scoring alone."""
    gp = _gp()
    from paper_2607_06731_amd import synth
    rng = np.random.default_rng(77)
    runs = []
    for n in (33 * 256 - 5, 32 * 256 - 7, 65 * 128 + 3):
        X = rng.standard_normal((3, n)).astype(np.float32)
        y = (X[0] * X[1] + rng.normal(0, 0.05, n)).astype(np.float32)
        runs.append(synth.ServingRun(len(runs), synth.Dataset(X, y)))
    reqs = [(i, synth.make_serving_request(rng, runs[i], min_pop=300, max_pop=600))
            for i in (0, 1, 2, 1)]
    _say("batched mixed tile counts")
    got = _run_batched(gp, runs, reqs, 1e-3)
    for (i, pop), (F, st) in zip(reqs, got):
        alone = gp.evaluate(pop.nodes, pop.offsets, pop.consts, runs[i].data.X, runs[i].data.y,
                            1e-3, 0)
        assert (st == 0).all()
        assert np.array_equal(F, alone, equal_nan=True)
