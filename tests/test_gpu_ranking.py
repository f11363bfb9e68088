"""gp_mc_rank (Monte-Carlo ranking, Table 2) against the ranking oracle:
integer work, so bands, children and the sorted sample must be bit-exact."""
import sys

import numpy as np
import pytest

from oracle import ranking

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


def _rank_gpu(gp, f, higher, seed, S):
    import torch
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    band = torch.full((f.size,), -1, dtype=torch.int32, device="cuda")
    ch = torch.full((f.size,), -1.0, dtype=torch.float32, device="cuda")
    keys = torch.empty(S, dtype=torch.float64, device="cuda")
    gp.gp_mc_rank(ft, higher, seed, band, ch, keys, sample_size=S)
    torch.cuda.synchronize()
    return band.cpu().numpy(), ch.cpu().numpy(), keys.cpu().numpy()


def _fitness(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)
    f[rng.random(n) < 0.02] = np.nan
    f[rng.random(n) < 0.02] = np.inf
    f[rng.random(n) < 0.05] = 1.25             # ties
    return f


@pytest.mark.parametrize("n,S,higher,seed", [(1, 100, False, 0), (7, 100, True, 3),
                                             (1000, 100, False, 42), (1000, 1, True, 5),
                                             (1 << 20, 100, False, 2026),
                                             (300_000, 1024, True, 77)])
def test_rank_matches_oracle(n, S, higher, seed):
    gp = _gp()
    f = _fitness(n, seed)
    _say("mc rank n=%d S=%d higher=%s seed=%d" % (n, S, higher, seed))
    b, c, k = _rank_gpu(gp, f, higher, seed, S)
    rb, rc, rk = ranking.mc_rank(f, higher, seed, S)
    assert np.array_equal(b, rb)
    assert np.array_equal(c, rc)
    assert np.array_equal(k, rk)


def test_rank_of_scored_population():
    """The step after scoring: rank gp_eval's output on the device."""
    gp = _gp()
    import torch
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=20000, n_cases=1024)
    F = gp.evaluate(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X, w.data.y, w.tax,
                    w.allowed_mask)
    b, c, k = _rank_gpu(gp, F, False, 99, 100)
    rb, rc, rk = ranking.mc_rank(F, False, 99, 100)
    _say("mc rank of a scored population: mean children %.3f" % c.mean())
    assert np.array_equal(b, rb) and np.array_equal(c, rc)
    assert 0.7 < c.mean() < 1.3
