"""CPU-side checks of the C ABI: the library loads, exports every function
that include/gpeval.h declares, validates on the host exactly like the
oracle's independent validator, and rejects bad arguments synchronously
(before any device work)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2607_06731_amd as gp
from paper_2607_06731_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(gp_\w+)\s*\(", text, re.M):
            names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(gp.LIB_PATH):
        from paper_2607_06731_amd import _build
        _build.build()
    return gp.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "gp_eval" in names and "gp_validate" in names
    for n in names:
        assert hasattr(L, n), n


def test_version(L):
    assert L.gp_version() >= 1


def test_host_validate_matches_oracle_on_brute_force():
    from tests.test_oracle_pins import brute_force_programs
    seqs = brute_force_programs(4)
    lens = np.array([len(s) for s in seqs], np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([t for s in seqs for t in s], np.uint32)
    st_o, md_o = oracle.validate(nodes, off, 1, 2, oracle.MASK_BENCH)
    st_g, md_g, first = gp.gp_validate(nodes, off, 1, 2, gp.GP_ALL_OPS)
    assert np.array_equal(st_o == 0, st_g == 0)
    assert np.array_equal(md_o[st_o == 0], md_g[st_g == 0])


def test_host_validate_status_codes():
    rng = np.random.default_rng(1)
    w = synth.make_workload("generation", n_programs=2000, n_cases=64)
    nodes = w.pop.nodes.copy()
    # mutate: random opcodes, operand indices and truncations
    idx = rng.choice(nodes.size, 300, replace=False)
    nodes[idx[:100]] = rng.integers(0, 16, 100).astype(np.uint32)
    nodes[idx[100:200]] = (nodes[idx[100:200]] & 0xFF) | (rng.integers(0, 9, 100).astype(np.uint32) << 8)
    st_o, _ = oracle.validate(nodes, w.pop.offsets, w.pop.consts.size, 5, w.allowed_mask)
    st_g, _, first = gp.gp_validate(nodes, w.pop.offsets, w.pop.consts.size, 5, w.allowed_mask)
    assert np.array_equal(st_o, st_g)
    bad = np.nonzero(st_g)[0]
    assert first == (bad[0] if bad.size else -1)


def test_eval_rejects_bad_arguments_before_device_work(L):
    c = ctypes.c_void_p(1)   # never dereferenced: checks fail first
    # negative sizes
    assert L.gp_eval(c, c, -1, 0, c, 0, c, 1, 1, c, 1, 0.0, 0, c, None, None) == gp.GP_E_INVALID_ARG
    assert L.gp_eval(c, c, 1, 1, c, 0, c, 1, 1, c, 0, 0.0, 0, c, None, None) == gp.GP_E_INVALID_ARG
    # ld_x < n_cases
    assert L.gp_eval(c, c, 1, 1, c, 0, c, 1, 10, c, 11, 0.0, 0, c, None, None) == gp.GP_E_INVALID_ARG
    # too many constants for a 24-bit operand
    assert L.gp_eval(c, c, 1, 1, c, 1 << 25, c, 1, 10, c, 10, 0.0, 0, c, None, None) == gp.GP_E_TOO_LARGE
    assert b"n_consts" in L.gp_last_error()
    # empty population is a no-op
    assert L.gp_eval(None, c, 0, 0, None, 0, None, 0, 1, c, 1, 0.0, 0, None, None, None) == gp.GP_OK


def test_noalloc_rejects_bad_arguments_before_device_work(L):
    """gp_eval_noalloc checks its arguments as gp_eval does, before it takes
    the fixed workspace's device address."""
    c = ctypes.c_void_p(1)
    f = L.gp_eval_noalloc
    assert f(c, c, -1, 0, c, 0, c, 1, 1, c, 1, 0.0, 0, c, None, None) == gp.GP_E_INVALID_ARG
    assert f(c, c, 1, 1, c, 0, c, 1, 10, c, 11, 0.0, 0, c, None, None) == gp.GP_E_INVALID_ARG
    assert f(c, c, 1, 1, c, 1 << 25, c, 1, 10, c, 10, 0.0, 0, c, None, None) == gp.GP_E_TOO_LARGE
    assert f(c, c, 1, 1, c, 0, c, 1, 1, c, 1, 0.0, 1 << 28, c, None, None) == gp.GP_E_INVALID_ARG
    assert f(None, c, 0, 0, None, 0, None, 0, 1, c, 1, 0.0, 0, None, None, None) == gp.GP_OK


def test_correlation_rejects_bad_arguments_before_device_work(L):
    c = ctypes.c_void_p(1)
    for M in (float("nan"), float("inf")):
        assert L.gp_eval_correlation(c, c, 1, 1, c, 0, c, 1, 1, c, 1, M, 0, c, None,
                                     None) == gp.GP_E_INVALID_ARG
        assert b"max_score" in L.gp_last_error()
    assert L.gp_eval_correlation(c, c, -1, 0, c, 0, c, 1, 1, c, 1, 1e4, 0, c, None,
                                 None) == gp.GP_E_INVALID_ARG
    assert L.gp_eval_correlation(None, c, 0, 0, None, 0, None, 0, 1, c, 1, 1e4, 0, None,
                                 None, None) == gp.GP_OK


def test_reward_rejects_bad_arguments_before_device_work(L):
    c = ctypes.c_void_p(1)
    for M in (float("nan"), float("inf"), -float("inf"), 2.0 ** 24 + 2.0, 7.75, -0.5):
        assert L.gp_eval_reward(c, c, 1, 1, c, 0, c, 1, 1, c, 1, M, 1, 0, c, None,
                                None) == gp.GP_E_INVALID_ARG
        assert b"max_score" in L.gp_last_error()
    for power in (0, 4, 5, -1, 16):
        assert L.gp_eval_reward(c, c, 1, 1, c, 0, c, 1, 1, c, 1, 1e4, power, 0, c, None,
                                None) == gp.GP_E_INVALID_ARG
        assert b"power" in L.gp_last_error()
    assert L.gp_eval_reward(c, c, -1, 0, c, 0, c, 1, 1, c, 1, 1e4, 2, 0, c, None,
                            None) == gp.GP_E_INVALID_ARG
    for power in (1, 2, 3, 8):
        assert L.gp_eval_reward(None, c, 0, 0, None, 0, None, 0, 1, c, 1, 1e4, power, 0, None,
                                None, None) == gp.GP_OK


def test_scoring_rejects_masks_beyond_the_command_table(L):
    c = ctypes.c_void_p(1)
    for mask in (1 << 28, gp.GP_ALL_OPS | (1 << 31), gp.GP_BASE_OPS | (1 << 29)):
        assert L.gp_eval(c, c, 1, 1, c, 0, c, 1, 1, c, 1, 0.0, mask, c, None,
                         None) == gp.GP_E_INVALID_ARG
        assert b"GP_ALL_OPS" in L.gp_last_error()
        assert L.gp_eval_correlation(c, c, 1, 1, c, 0, c, 1, 1, c, 1, 1e4, mask, c, None,
                                     None) == gp.GP_E_INVALID_ARG
        assert L.gp_eval_reward(c, c, 1, 1, c, 0, c, 1, 1, c, 1, 1e4, 1, mask, c, None,
                                None) == gp.GP_E_INVALID_ARG


def test_binding_refuses_host_tensors():
    import torch
    with pytest.raises(TypeError):
        gp._dev_ptr(torch.zeros(3, dtype=torch.float32), torch.float32, "x")


def test_no_oracle_in_product_path():
    # the product package must not import or reference the oracle
    pkg = os.path.join(ROOT, "paper_2607_06731_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "gp_oracle" not in text, fn


def test_workspace_size_model(L):
    ws = gp.workspace_size
    base = ws(0, 0)
    assert ws(1000, 0) > base and ws(0, 100000) > base
    # more programs and nodes never need less
    assert ws(2000, 50000) >= ws(1000, 50000) >= ws(1000, 40000)
    # more cases means more tiles per program (at most 32)
    assert ws(1000, 0, max_n_cases=1 << 20) > ws(1000, 0, max_n_cases=1024)
    assert ws(1000, 0, max_n_cases=1 << 30) == ws(1000, 0, max_n_cases=1 << 20)
    b = ctypes.c_size_t()
    assert L.gp_workspace_size(-1, 0, 1, 1, 1, 1, ctypes.byref(b)) == gp.GP_E_INVALID_ARG
    assert L.gp_workspace_size(1, 0, 0, 1, 1, 1, ctypes.byref(b)) == gp.GP_E_INVALID_ARG


def test_batched_and_server_reject_bad_arguments(L):
    c = ctypes.c_void_p(1)
    # NULL tables / counts < 1 fail before any device work
    assert L.gp_eval_batched(None, 1, c, 1, 1, 1, 1, 1, 0, None) == gp.GP_E_INVALID_ARG
    assert L.gp_eval_batched(c, 1, None, 1, 1, 1, 1, 1, 0, None) == gp.GP_E_INVALID_ARG
    assert L.gp_eval_batched(c, 0, c, 1, 1, 1, 1, 1, 0, None) == gp.GP_E_INVALID_ARG
    assert L.gp_eval_batched(c, 5000, c, 1, 1, 1, 1, 1, 0, None) == gp.GP_E_TOO_LARGE
    h = ctypes.c_void_p()
    cfg = gp.GPServerConfig(1 << 20, 0, 0, 0, 0, 0, 0, 0)          # budget below 16 MiB
    assert L.gp_server_create(ctypes.byref(h), ctypes.byref(cfg)) == gp.GP_E_INVALID_ARG
    cfg = gp.GPServerConfig(0, 0, 0, 0, 9, 0, 0, 0)                # too many streams
    assert L.gp_server_create(ctypes.byref(h), ctypes.byref(cfg)) == gp.GP_E_INVALID_ARG
    t = ctypes.c_int64()
    assert L.gp_server_submit(None, 0, None, 0, c, 0, None, 0, None, None,
                              ctypes.byref(t)) == gp.GP_E_INVALID_ARG


def test_host_validate_matches_oracle_on_the_full_command_table():
    """Status codes and maximum depth (stack plus held variables) of the
    host validator equal the oracle's over every program of up to five
    tokens of an alphabet with the stack moves, variables and POW, and over
    mutated programs of the GCL workload."""
    import itertools
    from oracle import COPY, DEL, DUP, PASTE, POW, SWAP
    L0, C0 = oracle.LOAD, oracle.CONST
    alphabet = [L0, C0, oracle.SIN, oracle.ADD, POW, DUP, SWAP, DEL, COPY, PASTE,
                COPY | (1 << 8), PASTE | (1 << 8), COPY | (16 << 8), 28]
    progs = [t for n in range(1, 5) for t in itertools.product(alphabet, repeat=n)]
    lens = np.array([len(p) for p in progs], np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    nodes = np.array([w for p in progs for w in p], np.uint32)
    st_o, md_o = oracle.validate(nodes, off, 1, 1, oracle.MASK_GCL)
    st_g, md_g, _ = gp.gp_validate(nodes, off, 1, 1, gp.GP_ALL_OPS)
    assert np.array_equal(st_o, st_g)
    ok = st_o == 0
    assert ok.sum() > 100 and np.array_equal(md_o[ok], md_g[ok])
    # a mask without the moves rejects them
    st_b, _, _ = gp.gp_validate(nodes, off, 1, 1, gp.GP_BASE_OPS)
    st_ob, _ = oracle.validate(nodes, off, 1, 1, oracle.MASK_BENCH)
    assert np.array_equal(st_b, st_ob)
    w = synth.make_workload("gcl", n_programs=2000, n_cases=64)
    rng = np.random.default_rng(3)
    nodes = w.pop.nodes.copy()
    idx = rng.choice(nodes.size, 400, replace=False)
    nodes[idx[:200]] = rng.integers(0, 30, 200).astype(np.uint32)
    nodes[idx[200:]] = (nodes[idx[200:]] & 0xFF) | (rng.integers(0, 18, 200).astype(np.uint32) << 8)
    st_o, md_o = oracle.validate(nodes, w.pop.offsets, w.pop.consts.size, 4, w.allowed_mask)
    st_g, md_g, _ = gp.gp_validate(nodes, w.pop.offsets, w.pop.consts.size, 4, w.allowed_mask)
    assert np.array_equal(st_o, st_g)
    ok = st_o == 0
    assert np.array_equal(md_o[ok], md_g[ok])
    assert (st_o == oracle.ST_BAD_PAIR).sum() > 10
