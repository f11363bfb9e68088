"""Plans (captured hipGraph of the whole pipeline, autotuned scheduling):
results are bit-identical to gp_eval whatever the tuning, relaunches see
in-place buffer updates, and updates re-capture for new sizes."""
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
                   {"programs_per_item": 4, "concurrent_classes": 1}):
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
    assert np.array_equal(F1, F_ref, equal_nan=True)
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
        assert np.array_equal(F2, F2_ref, equal_nan=True)
    # different size: update re-captures
    w3 = synth.make_workload("generation", n_programs=11111, n_cases=4096, seed=78)
    pop3 = gp.DevicePopulation(w3.pop.nodes, w3.pop.offsets, w3.pop.consts)
    out3 = torch.empty(pop3.n_programs, dtype=torch.float64, device="cuda")
    plan.update(pop3, data, w.tax, out3, allowed_op_mask=w.allowed_mask)
    plan.launch()
    torch.cuda.synchronize()
    F3_ref = gp.evaluate(w3.pop.nodes, w3.pop.offsets, w3.pop.consts, w.data.X, w.data.y,
                         w.tax, w.allowed_mask)
    assert np.array_equal(out3.cpu().numpy(), F3_ref, equal_nan=True)
    plan.close()
