"""Host builds under AddressSanitizer and UndefinedBehaviorSanitizer: the
fp64 oracle (through tests/oracle_driver.c) and the library's staging walk
(tests/staging_harness.cpp) run on workloads with every command of the
table, invalid programs and non-finite data; any sanitizer report fails the
run (-fno-sanitize-recover), and the results equal the normal builds' bit
for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2607_06731_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]


def _need(tool):
    exe = shutil.which(tool)
    if not exe:
        pytest.skip("no host compiler " + tool)
    return exe


def _populations():
    rng = np.random.default_rng(12)
    out = []
    w = synth.make_workload("gcl", n_programs=600, n_cases=40)
    nodes = w.pop.nodes.copy()
    idx = rng.choice(nodes.size, 60, replace=False)
    nodes[idx[:30]] = rng.integers(0, 30, 30).astype(np.uint32)        # bad opcodes
    nodes[idx[30:]] = (nodes[idx[30:]] & 0xFF) | (rng.integers(0, 18, 30).astype(np.uint32) << 8)
    y = w.data.y.copy()
    y[::11] = np.nan
    y[5::13] = np.inf
    out.append((nodes, w.pop.offsets, w.pop.consts, w.data.X, y, oracle.MASK_GCL))
    g = synth.make_workload("generation", n_programs=800, n_cases=64)
    X = g.data.X.copy()
    X[0, ::9] = np.inf
    X[1, 3::17] = np.nan
    out.append((g.pop.nodes, g.pop.offsets, g.pop.consts, X, g.data.y, oracle.MASK_BENCH))
    return out


def _write(path, nodes, offsets, consts, X, y=None):
    nodes = np.ascontiguousarray(nodes, np.uint32)
    offsets = np.ascontiguousarray(offsets, np.int64)
    consts = np.ascontiguousarray(consts, np.float32)
    X = np.ascontiguousarray(X, np.float32)
    with open(path, "wb") as f:
        np.array([offsets.size - 1, nodes.size, consts.size, X.shape[0], X.shape[1]],
                 np.int64).tofile(f)
        nodes.tofile(f)
        offsets.tofile(f)
        consts.tofile(f)
        X.tofile(f)
        if y is not None:
            np.ascontiguousarray(y, np.float32).tofile(f)


def test_oracle_under_asan_ubsan(tmp_path):
    cc = _need("gcc")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call([cc, "-O1", "-std=c11", "-pthread", "-ffp-contract=off"] + SAN +
                          [os.path.join(ROOT, "tests", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "gp_oracle.c"), "-lm", "-o", exe])
    for k, (nodes, offsets, consts, X, y, mask) in enumerate(_populations()):
        fin, fout = str(tmp_path / ("in%d" % k)), str(tmp_path / ("out%d" % k))
        _write(fin, nodes, offsets, consts, X, y)
        r = subprocess.run([exe, fin, fout, str(mask)], capture_output=True, text=True)
        assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-3000:]
        P = offsets.size - 1
        raw = np.fromfile(fout, np.uint8)
        st = raw[:4 * P].view(np.int32)
        md = raw[4 * P:8 * P].view(np.int32)
        vals = raw[8 * P:8 * P + 48 * P].view(np.float64).reshape(6, P)
        c12 = raw[8 * P + 48 * P:].view(np.int64).reshape(P, 2)
        st_o, md_o = oracle.validate(nodes, offsets, consts.size, X.shape[0], mask)
        assert np.array_equal(st, st_o) and np.array_equal(md, md_o)
        F, mse, _ = oracle.fitness(nodes, offsets, consts, X, y, 1e-3, mask)
        F17, _, _ = oracle.fitness(nodes, offsets, consts, X, y, 1e-3, mask, oracle.M32E_RAND + 1)
        S, r, _, c1, c2 = oracle.correlation(nodes, offsets, consts, X, y, 1e4, mask,
                                             return_counts=True)
        R, _ = oracle.reward(nodes, offsets, consts, X, y, 1e4, 8, mask)
        for got, ref in ((vals[0], F), (vals[1], F17), (vals[2], mse), (vals[3], S),
                         (vals[4], r), (vals[5], R)):
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)) or \
                np.array_equal(got, ref, equal_nan=True)
        ok = st_o == 0
        assert np.array_equal(c12[ok, 0], c1[ok]) and np.array_equal(c12[ok, 1], c2[ok])


def test_staging_walk_under_asan_ubsan(tmp_path):
    cxx = _need("g++")
    exe = str(tmp_path / "staging_san")
    subprocess.check_call([cxx, "-O1", "-std=c++17", "-ffp-contract=off",
                           "-D__HIP_PLATFORM_AMD__"] + SAN +
                          ["-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2607_06731_amd", "csrc"),
                           "-I", "/opt/rocm/include",
                           os.path.join(ROOT, "tests", "staging_harness.cpp"), "-o", exe])
    from tests.test_staging_host import _run as run_harness
    plain = None
    for k, (nodes, offsets, consts, X, y, mask) in enumerate(_populations()):
        X = np.nan_to_num(X, nan=0.5, posinf=2.0)
        info, out = run_harness(exe, tmp_path, nodes, offsets, consts, X)
        st_o, _ = oracle.validate(nodes, offsets, consts.size, X.shape[0], oracle.MASK_GCL)
        assert np.array_equal(info[:, 0], st_o)
        ok = st_o == 0
        assert np.array_equal(info[ok, 2], info[ok, 3]) and np.all(info[ok, 4] == 1)
