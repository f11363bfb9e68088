"""gp_eval_noalloc: gp_eval on the library's fixed device workspace.

Its results must equal gp_eval's bit for bit (the same kernels and the same
summation order), on two calls in a row, the second with a smaller input
(the fixed array keeps the first call's contents); the smaller call is also
gated against the fp64 oracle.  A call needing more workspace than the
array holds is rejected before any device work.
"""
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


def _both(gp, w):
    import torch
    pop = gp.DevicePopulation(w.pop.nodes, w.pop.offsets, w.pop.consts)
    data = gp.DeviceDataset(w.data.X, w.data.y)
    P = pop.n_programs
    a = torch.full((P,), -1.0, dtype=torch.float64, device="cuda")
    b = torch.full((P,), -2.0, dtype=torch.float64, device="cuda")
    sa = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    sb = torch.full((P,), -8, dtype=torch.int32, device="cuda")
    gp.gp_eval(pop.nodes, pop.offsets, pop.consts, data.X, data.y, w.tax, a, sa,
               w.allowed_mask)
    gp.gp_eval_noalloc(pop.nodes, pop.offsets, pop.consts, data.X, data.y, w.tax, b, sb,
                       w.allowed_mask)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), sa.cpu().numpy(), sb.cpu().numpy()


def test_noalloc_equals_gp_eval_on_two_calls():
    gp = _gp()
    from paper_2607_06731_amd import synth
    for name, P, n in (("generation", 30000, 4096), ("generation", 3000, 1025)):
        w = synth.make_workload(name, n_programs=P, n_cases=n)
        _say("noalloc vs gp_eval: %s P=%d n=%d" % (name, P, n))
        Fa, Fb, sa, sb = _both(gp, w)
        assert np.array_equal(sa, sb)
        assert np.array_equal(Fa.view(np.uint64), Fb.view(np.uint64))
    rep = gate.check(Fb, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
                     w.allowed_mask)
    _say("noalloc second call vs oracle: " + rep.summary())
    assert rep.ok(), rep.failures[:5]


def test_noalloc_rejects_a_call_beyond_the_array():
    gp = _gp()
    import torch
    L = gp.lib()
    need = int(gp.GP_NOALLOC_WORKSPACE_BYTES) // 8 + 1      # nodes whose staged code alone is too big
    t = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = t.data_ptr()
    _say("noalloc size limit")
    # sizes are checked before any device work; no pointer is dereferenced
    rc = L.gp_eval_noalloc(p, p, 1, need, p, 0, p, 1, 16, p, 16, 0.0, 0, p, None, None)
    assert rc == gp.GP_E_TOO_LARGE
    assert b"fixed array" in L.gp_last_error()
