"""Plans (captured hipGraph of the whole pipeline, autotuned launch knobs):
with the default tile knobs results are bit-identical to gp_eval whatever
the other knobs; other tile knobs (window budget, tiles per program) give
deterministic results that pass the oracle's gate; relaunches see in-place
buffer updates, and updates re-capture for new sizes; the autotuned plan of
the uneven workload at full size is gated against the oracle."""
import sys

import numpy as np
import pytest

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


def _close(a, b):
    """Same classes, and finite values within 1e-5 relative (another
    summation grouping of the same compensated sums)."""
    fa, fb = np.isfinite(a), np.isfinite(b)
    if not (np.array_equal(fa, fb) and np.array_equal(np.isnan(a), np.isnan(b))):
        return False
    return bool(np.all(np.abs(a[fa] - b[fa]) <= 1e-5 * np.abs(b[fa]) + 1e-12))


def test_plan_matches_eval_for_every_tuning():
    gp = _gp()
    import torch
    from paper_2607_06731_amd import synth
    w = synth.make_workload("uneven", n_programs=20000, n_cases=3000)
    pop = gp.DevicePopulation(w.pop.nodes, w.pop.offsets, w.pop.consts)
    data = gp.DeviceDataset(w.data.X, w.data.y)
    ref = torch.empty(pop.n_programs, dtype=torch.float64, device="cuda")
    _say("plan vs eval")
    gp.gp_eval(pop.nodes, pop.offsets, pop.consts, data.X, data.y, w.tax, ref,
               allowed_op_mask=w.allowed_mask)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    for tuning in ({"programs_per_item": 1}, {"programs_per_item": 32, "wg_per_cu": 2},
                   {"programs_per_item": 128},
                   {"programs_per_item": 4, "concurrent_classes": 1},
                   {"programs_per_item": 64, "concurrent_classes": 2}):
        out = torch.full((pop.n_programs,), -1.0, dtype=torch.float64, device="cuda")
        plan = gp.Plan(pop, data, w.tax, out, allowed_op_mask=w.allowed_mask, tuning=tuning)
        for _ in range(3):          # replays with host work in between
            plan.launch()
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got, ref, equal_nan=True), tuning
        plan.close()


def test_plan_autotune_and_inplace_update():
    gp = _gp()
    import torch
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=30000, n_cases=4096)
    pop = gp.DevicePopulation(w.pop.nodes, w.pop.offsets, w.pop.consts)
    data = gp.DeviceDataset(w.data.X, w.data.y)
    out = torch.empty(pop.n_programs, dtype=torch.float64, device="cuda")
    _say("plan autotune")
    plan = gp.Plan(pop, data, w.tax, out, allowed_op_mask=w.allowed_mask, autotune=True)
    t = plan.tuning
    assert 1 <= t["programs_per_item"] <= 128
    plan.launch()
    torch.cuda.synchronize()
    F1 = out.cpu().numpy()
    F_ref = gp.evaluate(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
                        w.allowed_mask)
    _say("tuning %s" % t)
    default_tiles = t["tile_lds_bytes"] == 24576 and t["max_tiles"] == 32
    agree = (lambda a, b: np.array_equal(a, b, equal_nan=True)) if default_tiles else _close
    assert agree(F1, F_ref)
    # next generation: same shape, new programs written in place
    w2 = synth.make_workload("generation", n_programs=30000, n_cases=4096, seed=77)
    same = w2.pop.nodes.size == w.pop.nodes.size and w2.pop.consts.size == w.pop.consts.size
    if same:
        pop.nodes.copy_(torch.from_numpy(w2.pop.nodes).cuda())
        pop.offsets.copy_(torch.from_numpy(w2.pop.offsets).cuda())
        pop.consts.copy_(torch.from_numpy(w2.pop.consts).cuda())
        plan.launch()
        torch.cuda.synchronize()
        F2 = out.cpu().numpy()
        F2_ref = gp.evaluate(w2.pop.nodes, w2.pop.offsets, w2.pop.consts, w.data.X, w.data.y,
                             w.tax, w.allowed_mask)
        assert agree(F2, F2_ref)
    # different size: update re-captures
    w3 = synth.make_workload("generation", n_programs=11111, n_cases=4096, seed=78)
    pop3 = gp.DevicePopulation(w3.pop.nodes, w3.pop.offsets, w3.pop.consts)
    out3 = torch.empty(pop3.n_programs, dtype=torch.float64, device="cuda")
    plan.update(pop3, data, w.tax, out3, allowed_op_mask=w.allowed_mask)
    plan.launch()
    torch.cuda.synchronize()
    F3_ref = gp.evaluate(w3.pop.nodes, w3.pop.offsets, w3.pop.consts, w.data.X, w.data.y,
                         w.tax, w.allowed_mask)
    assert agree(out3.cpu().numpy(), F3_ref)
    plan.close()


def test_plan_replays_follow_offsets_written_in_place():
    """A plan derives its dataset and request tables once; each replay still
    follows the offsets as they are then: offsets rewritten to decrease
    somewhere (every program staged again, packed) and back (staged in
    place) give gp_eval's bits on every replay."""
    gp = _gp()
    import torch
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=20000, n_cases=1500)
    pop = gp.DevicePopulation(w.pop.nodes, w.pop.offsets, w.pop.consts)
    data = gp.DeviceDataset(w.data.X, w.data.y)
    out = torch.empty(pop.n_programs, dtype=torch.float64, device="cuda")
    _say("plan replays with offsets rewritten in place")
    plan = gp.Plan(pop, data, w.tax, out, allowed_op_mask=w.allowed_mask,
                   tuning={"concurrent_classes": 2})
    bad = w.pop.offsets.copy()
    bad[101] = bad[100] - 1                  # program 100 ends before it starts
    for off in (w.pop.offsets, bad, w.pop.offsets, bad):
        pop.offsets.copy_(torch.from_numpy(off).cuda())
        plan.launch()
        torch.cuda.synchronize()
        ref, st = gp.evaluate(w.pop.nodes, off, w.pop.consts, w.data.X, w.data.y, w.tax,
                              w.allowed_mask, return_status=True)
        assert np.array_equal(out.cpu().numpy(), ref, equal_nan=True)
        assert (st[100] == 8) == (off is bad)
    plan.close()


def test_tile_knobs_deterministic_and_gated():
    """Window budgets and tile caps other than gp_eval's group the cases
    differently: every replay gives the same bits, and the results pass the
    oracle's gate."""
    gp = _gp()
    import torch
    from oracle import gate
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=3000, n_cases=5000)
    pop = gp.DevicePopulation(w.pop.nodes, w.pop.offsets, w.pop.consts)
    data = gp.DeviceDataset(w.data.X, w.data.y)
    for tuning in ({"tile_lds_bytes": 12288, "max_tiles": 2},
                   {"tile_lds_bytes": 40960, "max_tiles": 8, "programs_per_item": 32},
                   {"max_tiles": 1}):
        out = torch.full((pop.n_programs,), -1.0, dtype=torch.float64, device="cuda")
        plan = gp.Plan(pop, data, w.tax, out, allowed_op_mask=w.allowed_mask, tuning=tuning)
        plan.launch()
        torch.cuda.synchronize()
        first = out.cpu().numpy()
        for _ in range(2):
            plan.launch()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), first, equal_nan=True)
        assert plan.tuning["max_tiles"] == tuning["max_tiles"]
        plan.close()
        rep = gate.check(first, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y,
                         w.tax, w.allowed_mask)
        _say("tiles %s: %s" % (tuning, rep.summary()))
        assert rep.ok(), rep.failures[:5]


def test_uneven_autotuned_plan_full_size_gated():
    """The uneven workload at full size (1,000,000 programs x 16,384 cases)
    through an autotuned plan, gated against the oracle on a seeded sample
    stratified by length."""
    gp = _gp()
    import time
    import torch
    from oracle import gate
    from paper_2607_06731_amd import synth
    w = synth.make_workload("uneven")
    pop = gp.DevicePopulation(w.pop.nodes, w.pop.offsets, w.pop.consts)
    data = gp.DeviceDataset(w.data.X, w.data.y)
    out = torch.full((pop.n_programs,), -1.0, dtype=torch.float64, device="cuda")
    _say("uneven plan autotune at full size")
    t0 = time.time()
    plan = gp.Plan(pop, data, w.tax, out, allowed_op_mask=w.allowed_mask, autotune=True)
    _say("tuned in %.1f s: %s" % (time.time() - t0, plan.tuning))
    plan.launch()
    torch.cuda.synchronize()
    F = out.cpu().numpy()
    plan.close()
    assert not np.isnan(F).any()
    rng = np.random.default_rng(45)
    L = w.pop.lengths
    idx = []
    for l in np.unique(L):
        pool = np.nonzero(L == l)[0]
        idx.append(rng.choice(pool, min(4, pool.size), replace=False))
    idx = rng.permutation(np.concatenate(idx))[:400]
    sub = w.pop.take(idx)
    rep = gate.check(F[idx], sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y, w.tax,
                     w.allowed_mask)
    _say("uneven plan (sampled %d): %s" % (idx.size, rep.summary()))
    assert rep.ok(), rep.failures[:5]
