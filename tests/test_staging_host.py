"""The library's staging walk on the host (paper_2607_06731_amd/csrc/
staging.h, built into tests/staging_harness.cpp with the host compiler):
the validator's status and maximum depth equal the oracle's, the staged
instruction count equals what the walk emits, the end flag sits on the last
word only, no program outgrows its node count, and the staged words,
evaluated by the harness's plain evaluator, give the oracle's fp32-mode
values (bit for bit for the commands whose fp32 result is one rounding,
closely otherwise)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import ABS, ADD, DIV, MUL, SIGN, SQUARE, SUB, CUBE
from paper_2607_06731_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MASK = oracle.MASK_GCL


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("staging") / "staging_harness")
    subprocess.check_call([cxx, "-O1", "-std=c++17", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2607_06731_amd", "csrc"),
                           "-I", "/opt/rocm/include",
                           os.path.join(ROOT, "tests", "staging_harness.cpp"), "-o", exe])
    return exe


def _run(exe, tmp, nodes, offsets, consts, X):
    nodes = np.ascontiguousarray(nodes, np.uint32)
    offsets = np.ascontiguousarray(offsets, np.int64)
    consts = np.ascontiguousarray(consts, np.float32)
    X = np.ascontiguousarray(X, np.float32)
    P = offsets.size - 1
    n_vars, n_cases = X.shape
    fin, fout = str(tmp / "in.bin"), str(tmp / "out.bin")
    with open(fin, "wb") as f:
        np.array([P, nodes.size, consts.size, n_vars, n_cases], np.int64).tofile(f)
        nodes.tofile(f)
        offsets.tofile(f)
        consts.tofile(f)
        X.tofile(f)
    subprocess.check_call([exe, fin, fout])
    raw = np.fromfile(fout, np.uint8)
    info = raw[:P * 8 * 8].view(np.int64).reshape(P, 8)
    out = raw[P * 8 * 8:].view(np.float32).reshape(P, n_cases)
    # the benchmark-set walks agree with the general ones on every program
    assert info[:, 6].all(), np.nonzero(info[:, 6] == 0)[0][:10]
    assert info[:, 7].all(), np.nonzero(info[:, 7] == 0)[0][:10]
    return info, out


def _m32e(nodes, offsets, consts, X):
    return np.stack([oracle.program_outputs(nodes[offsets[i]:offsets[i + 1]], consts, X,
                                            allowed_mask=MASK, mode=oracle.M32E)
                     for i in range(offsets.size - 1)])


def _check_structure(info, nodes, offsets, n_consts, n_vars):
    st, md = oracle.validate(nodes, offsets, n_consts, n_vars, MASK)
    assert np.array_equal(info[:, 0], st)
    ok = st == 0
    assert np.array_equal(info[ok, 1], md[ok])
    assert np.array_equal(info[ok, 2], info[ok, 3])          # counted == emitted
    assert np.all(info[ok, 4] == 1)                           # end flag on the last word only
    assert np.all(info[ok, 5] == 1)                           # never more words than nodes
    return ok


def _bits_equal(a, b64):
    b = b64.astype(np.float32)
    return (a.view(np.uint32) == b.view(np.uint32)) | (np.isnan(a) & np.isnan(b))


def test_moves_and_single_rounding_commands_bit_exact(harness, tmp_path):
    rng = np.random.default_rng(3)
    pop = synth.sample_gcl_programs(rng, rng.integers(3, 49, 3000), 4,
                                    unary=(ABS, SQUARE, SIGN, CUBE), p_pow=0.0,
                                    binary=(ADD, SUB, MUL, DIV))
    X = rng.uniform(-2, 2, (4, 40)).astype(np.float32)
    info, out = _run(harness, tmp_path, pop.nodes, pop.offsets, pop.consts, X)
    ok = _check_structure(info, pop.nodes, pop.offsets, pop.consts.size, 4)
    assert ok.all()
    ref = _m32e(pop.nodes, pop.offsets, pop.consts, X)
    assert _bits_equal(out, ref).all()


def test_benchmark_set_and_long_constant_runs(harness, tmp_path):
    """Benchmark-set programs (folding across more than 16 held constants
    included) on the structure; the exact-op subset bit for bit."""
    rng = np.random.default_rng(4)
    pop = synth.sample_programs(rng, rng.integers(3, 65, 3000), 5, (ABS,),
                                binary=(ADD, SUB, MUL, DIV), p_var=0.15)
    X = rng.uniform(-3, 3, (5, 24)).astype(np.float32)
    info, out = _run(harness, tmp_path, pop.nodes, pop.offsets, pop.consts, X)
    assert _check_structure(info, pop.nodes, pop.offsets, pop.consts.size, 5).all()
    assert _bits_equal(out, _m32e(pop.nodes, pop.offsets, pop.consts, X)).all()
    # the generation workload's programs: structure and values
    w = synth.make_workload("generation", n_programs=2000, n_cases=24)
    info, out = _run(harness, tmp_path, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X)
    assert _check_structure(info, w.pop.nodes, w.pop.offsets, w.pop.consts.size, 5).all()
    ref = _m32e(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X)
    _close_or_ill_conditioned(out, ref, w, w.data.X)


def _close_or_ill_conditioned(out, ref, w, X):
    """Host library functions are not the device's: values must be close,
    except in programs whose fp32 and fp64 evaluations already differ."""
    fin = np.isfinite(ref)
    same_class = np.isfinite(out) == fin
    close = ~fin | (np.abs(out - ref) <= 1e-3 * np.abs(ref) + 1e-3)
    bad = np.nonzero(~(same_class & close).all(axis=1))[0]
    for p in bad:
        prog = w.pop.nodes[w.pop.offsets[p]:w.pop.offsets[p + 1]]
        o64 = oracle.program_outputs(prog, w.pop.consts, X, allowed_mask=MASK, mode=oracle.M64)
        up = oracle.program_outputs(prog, w.pop.consts, X, allowed_mask=MASK, mode=oracle.M32E_UP)
        sens = np.nanmax(np.abs(up - ref[p]) / np.maximum(np.abs(ref[p]), 1e-30))
        cls64 = np.isfinite(o64) != fin[p]
        assert sens > 1e-3 or cls64.any() or not np.isfinite(up).all(), int(p)
    assert bad.size <= 0.01 * out.shape[0]


def test_gcl_workload(harness, tmp_path):
    w = synth.make_workload("gcl", n_programs=4000, n_cases=16)
    info, out = _run(harness, tmp_path, w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X)
    assert _check_structure(info, w.pop.nodes, w.pop.offsets, w.pop.consts.size, 4).all()
    ref = _m32e(w.pop.nodes, w.pop.offsets, w.pop.consts, w.data.X)
    _close_or_ill_conditioned(out, ref, w, w.data.X)


def test_invalid_programs_get_the_oracle_status(harness, tmp_path):
    rng = np.random.default_rng(5)
    w = synth.make_workload("gcl", n_programs=1500, n_cases=4)
    nodes = w.pop.nodes.copy()
    idx = rng.choice(nodes.size, 300, replace=False)
    nodes[idx[:150]] = rng.integers(0, 30, 150).astype(np.uint32)
    nodes[idx[150:]] = (nodes[idx[150:]] & 0xFF) | (rng.integers(0, 18, 150).astype(np.uint32) << 8)
    info, _ = _run(harness, tmp_path, nodes, w.pop.offsets, w.pop.consts, w.data.X)
    ok = _check_structure(info, nodes, w.pop.offsets, w.pop.consts.size, 4)
    assert (~ok).sum() > 100


def test_benchmark_set_walk_on_invalid_programs(harness, tmp_path):
    """The one-pass benchmark-set walk names the same status as the general
    check on broken benchmark-set programs (opcodes out of the set or out of
    range, including the LDS copy's bad-constant byte, operands out of
    range, underflow, a stack too deep, a wrong final depth); _run asserts
    the agreement for every program under two masks."""
    rng = np.random.default_rng(6)
    w = synth.make_workload("generation", n_programs=3000, n_cases=4)
    nodes = w.pop.nodes.copy()
    offsets = w.pop.offsets.copy()
    idx = rng.choice(nodes.size, 600, replace=False)
    bytes_ = np.concatenate([rng.integers(0, 40, 200), [0x81, 0xFE, 0xFF] * 34])[:300]
    nodes[idx[:300]] = (nodes[idx[:300]] & ~np.uint32(0xFF)) | bytes_.astype(np.uint32)
    args = np.where(rng.random(300) < 0.5, rng.integers(0, 40, 300),
                    w.pop.consts.size + rng.integers(0, 40, 300))
    nodes[idx[300:]] = (nodes[idx[300:]] & 0xFF) | (args.astype(np.uint32) << 8)
    # programs cut short (wrong final depth, underflow in what follows)
    cut = rng.choice(offsets.size - 2, 200, replace=False) + 1
    offsets[cut] = offsets[cut] - rng.integers(0, 3, 200)
    offsets = np.maximum.accumulate(offsets)
    # stacks deeper than the limit: 40 leaves, then 39 additions
    deep = np.concatenate([np.full(40, oracle.CONST, np.uint32), np.full(39, ADD, np.uint32)])
    nodes = np.concatenate([nodes, deep, deep[:33], np.full(32, ADD, np.uint32)])
    offsets = np.concatenate([offsets, [offsets[-1] + 79, offsets[-1] + 79 + 65]])
    info, _ = _run(harness, tmp_path, nodes, offsets, w.pop.consts, w.data.X)
    st, _ = oracle.validate(nodes, offsets, w.pop.consts.size, 5, oracle.MASK_BENCH)
    seen = set(np.unique(st).tolist())
    assert {0, 2, 3, 4, 5, 6, 7} <= seen, seen
