"""gp_server: resident datasets, admission by device budget, chunking and
continuous batching.  Every served result must be bit-identical to gp_eval
of the same population alone; budgets, chunk sizes and stream counts are
scheduling choices that never change a result."""
import sys

import numpy as np
import pytest

import oracle

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


def _workload(n_req, seed, max_pop=2000, max_cases=8192, n_runs=4):
    from paper_2607_06731_amd import synth
    rng = np.random.default_rng(seed)
    runs = synth.make_serving_runs(n_runs, seed=seed, max_cases=max_cases)
    reqs = []
    for _ in range(n_req):
        i = int(rng.integers(0, len(runs)))
        reqs.append((i, synth.make_serving_request(rng, runs[i], min_pop=20, max_pop=max_pop)))
    return runs, reqs


def _alone(gp, runs, reqs, tax):
    return [gp.evaluate(p.nodes, p.offsets, p.consts, runs[i].data.X, runs[i].data.y, tax, 0)
            for i, p in reqs]


def _serve_all(srv, ids, reqs, timeout_s=60.0):
    import time
    tickets = {}
    for k, (i, p) in enumerate(reqs):
        tickets[srv.submit(ids[i], p.nodes, p.offsets, p.consts)] = k
    got = [None] * len(reqs)
    t0 = time.time()
    while any(g is None for g in got):
        assert time.time() - t0 < timeout_s, "requests did not complete"
        for t, rc, fit, st in srv.poll(timeout_ms=100.0):
            assert rc == 0
            got[tickets[t]] = (fit, st)
    return got


@pytest.mark.parametrize("mode", ["batched", "chunked", "one_per_request"])
def test_served_equals_alone(mode):
    gp = _gp()
    tax = 1e-3
    runs, reqs = _workload(24, seed=7)
    alone = _alone(gp, runs, reqs, tax)
    kw = {"device_budget_bytes": 256 << 20}
    if mode == "chunked":
        kw.update(chunk_node_evals=1 << 22, n_streams=3)
    if mode == "one_per_request":
        kw.update(one_launch_per_request=True)
    _say("server %s, %d requests" % (mode, len(reqs)))
    with gp.Server(**kw) as srv:
        ids = [srv.add_dataset(r.data.X, r.data.y, tax) for r in runs]
        got = _serve_all(srv, ids, reqs)
        stats = srv.stats()
    _say("stats %s" % {k: stats[k] for k in ("completed", "launches", "chunks_launched")})
    for (fit, st), ref in zip(got, alone):
        assert (st == 0).all()
        assert np.array_equal(fit, ref, equal_nan=True)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert 0 < stats["latency_p50_ms"] <= stats["latency_p99_ms"] <= stats["latency_max_ms"]
    if mode == "one_per_request":
        assert stats["launches"] == len(reqs)
    if mode == "chunked":
        assert stats["chunks_launched"] > len(reqs)
    if mode == "batched":
        assert stats["launches"] < len(reqs)      # submitted together: they share launches


def test_admission_under_small_budget():
    """A 16 MiB budget holds only a few requests at once: all still complete,
    the arena never overflows, and a request beyond the budget is refused."""
    gp = _gp()
    runs, reqs = _workload(30, seed=11, max_pop=3000, max_cases=4096, n_runs=2)
    alone = _alone(gp, runs, reqs, 0.0)
    _say("small budget")
    with gp.Server(device_budget_bytes=16 << 20, pinned_bytes=16 << 20) as srv:
        ids = [srv.add_dataset(r.data.X, r.data.y, 0.0) for r in runs]
        got = _serve_all(srv, ids, reqs)
        stats = srv.stats()
        assert stats["device_bytes_peak"] <= 12 << 20
        big = np.zeros(4 << 20, np.uint32)                # 16 MiB of nodes
        with pytest.raises(gp.GPError) as e:
            srv.submit(ids[0], big, np.array([0, big.size], np.int64), np.zeros(0, np.float32))
        assert e.value.code == gp.GP_E_TOO_LARGE
    for (fit, _), ref in zip(got, alone):
        assert np.array_equal(fit, ref, equal_nan=True)


def test_invalid_programs_and_dataset_lifetime():
    gp = _gp()
    runs, reqs = _workload(2, seed=13, max_pop=200, max_cases=1024, n_runs=1)
    i, pop = reqs[0]
    nodes = pop.nodes.copy()
    nodes[pop.offsets[3]] = oracle.LOAD | (999 << 8)       # variable out of range
    with gp.Server(device_budget_bytes=64 << 20) as srv:
        d = srv.add_dataset(runs[0].data.X, runs[0].data.y, 0.0)
        t = srv.submit(d, nodes, pop.offsets, pop.consts)
        # the dataset cannot go while a request on it is pending: a removal
        # that succeeds implies the request had already completed
        try:
            srv.remove_dataset(d)
            removed = True
        except gp.GPError as e:
            assert e.code == gp.GP_E_INVALID_ARG
            removed = False
        res = srv.wait(t, timeout_ms=0.0 if removed else 30000.0)
        assert res is not None
        rc, fit, st = res
        assert rc == 0 and st[3] == oracle.ST_BAD_VAR and np.isnan(fit[3])
        ok = np.setdiff1d(np.arange(fit.size), [3])
        ref = gp.evaluate(nodes, pop.offsets, pop.consts, runs[0].data.X, runs[0].data.y, 0.0, 0)
        assert np.array_equal(fit[ok], ref[ok], equal_nan=True)
        if not removed:
            srv.remove_dataset(d)
        with pytest.raises(gp.GPError):
            srv.submit(d, pop.nodes, pop.offsets, pop.consts)
        # empty population completes at once
        d2 = srv.add_dataset(runs[0].data.X, runs[0].data.y, 0.0)
        t2 = srv.submit(d2, np.zeros(0, np.uint32), np.zeros(1, np.int64), np.zeros(0, np.float32))
        rc2, fit2, _ = srv.wait(t2, timeout_ms=30000.0)
        assert rc2 == 0 and fit2.size == 0


def test_cancellation():
    """Requests cancelled while waiting or in flight complete with
    GP_E_CANCELLED and their output arrays are never written; the others
    still equal gp_eval alone; a completed ticket cannot be cancelled."""
    gp = _gp()
    import time
    runs, reqs = _workload(16, seed=17, max_pop=3000, max_cases=8192, n_runs=2)
    alone = _alone(gp, runs, reqs, 0.0)
    _say("cancellation")
    with gp.Server(device_budget_bytes=64 << 20, chunk_node_evals=1 << 22, n_streams=1) as srv:
        ids = [srv.add_dataset(r.data.X, r.data.y, 0.0) for r in runs]
        tickets = [srv.submit(ids[i], p.nodes, p.offsets, p.consts) for i, p in reqs]
        cancel = set()
        for t in tickets[1::3]:
            try:
                srv.cancel(t)
                cancel.add(t)
            except gp.GPError as e:          # it had completed already
                assert e.code == gp.GP_E_INVALID_ARG
        assert cancel
        got = {}
        t0 = time.time()
        while len(got) < len(tickets):
            assert time.time() - t0 < 60.0, "requests did not complete"
            for t, rc, fit, st in srv.poll(timeout_ms=100.0):
                got[t] = (rc, fit, st)
        with pytest.raises(gp.GPError) as e:
            srv.cancel(tickets[0])
        assert e.value.code == gp.GP_E_INVALID_ARG
        stats = srv.stats()
    for k, t in enumerate(tickets):
        rc, fit, st = got[t]
        if t in cancel:
            assert rc == gp.GP_E_CANCELLED
            assert np.all(fit == -1.0) and np.all(st == -1)
        else:
            assert rc == 0
            assert np.array_equal(fit, alone[k], equal_nan=True)
    assert stats["cancelled"] == len(cancel) and stats["completed"] == len(tickets) - len(cancel)
