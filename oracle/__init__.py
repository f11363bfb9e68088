"""CPU fp64 oracle for batched postfix-program fitness evaluation.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library.

``gp_oracle.c`` is the reference (plain interpreter, plain fp64 sums);
``tree_eval`` is a second, independent evaluator (recursive, over a parsed
expression tree, pure Python) used to cross-check it on brute-force sets;
``gcl`` parses the paper's textual GCL genomes.

Op numbering of the interchange format (node = op | arg << 8):
LOAD 0, CONST 1, ADD 2, SUB 3, MUL 4, DIV 5, SIN 6, COS 7, EXP 8, LOG 9,
SQRT 10, ABS 11; the rest of the GCL command table: DUP 12, SWAP 13, DEL 14,
SQUARE 15, SIGN 16, CUBE 17, CBRT 18, TAN 19, ARCSIN 20, ARCCOS 21, ARCTAN 22,
TANH 23, SQRT_RAW 24 (the paper's unprotected SQRT), POW 25, COPY 26, PASTE 27
(COPY/PASTE carry the variable name k < 16 in the arg field).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgp_oracle.so")

LOAD, CONST, ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, ABS = range(12)
DUP, SWAP, DEL, SQUARE = 12, 13, 14, 15
SIGN, CUBE, CBRT, TAN, ASIN, ACOS, ATAN, TANH, SQRT_RAW, POW, COPY, PASTE = range(16, 28)
N_OPS = 28

M64, M32E, M32E_UP, M32E_DN = 0, 1, 2, 3
M32E_RAND = 16      # M32E_RAND + seed: random +-2 ulp elementary functions

ST_VALID, ST_EMPTY, ST_BAD_OP, ST_BAD_VAR, ST_BAD_CONST = 0, 1, 2, 3, 4
ST_UNDERFLOW, ST_TOO_DEEP, ST_FINAL_DEPTH = 5, 6, 7
ST_BAD_PAIR = 10

#: every op of the benchmark set (LOAD..ABS)
MASK_BENCH = (1 << 12) - 1
#: the whole GCL command table (plus ABS)
MASK_GCL = (1 << N_OPS) - 1

THETA = float(np.float32(0.001))

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libgp_oracle.so``."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-pthread", "-fno-fast-math", "-ffp-contract=off",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        i64, i32, u32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
        L.oracle_check_program.argtypes = [vp, i64, i64, i32, u32, vp]
        L.oracle_check_program.restype = ctypes.c_int
        L.oracle_validate.argtypes = [vp, vp, i64, i64, i32, u32, vp, vp]
        L.oracle_validate.restype = None
        L.oracle_program_outputs.argtypes = [vp, i64, vp, i64, vp, i32, i64, i64,
                                             u32, ctypes.c_int, vp]
        L.oracle_program_outputs.restype = ctypes.c_int
        L.oracle_fitness.argtypes = [vp, vp, i64, vp, i64, vp, i32, i64, vp, i64,
                                     f64, u32, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.oracle_fitness.restype = ctypes.c_int
        L.oracle_correlation.argtypes = [vp, vp, i64, vp, i64, vp, i32, i64, vp, i64,
                                         f64, u32, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]
        L.oracle_correlation.restype = ctypes.c_int
        L.oracle_case_rewards.argtypes = [vp, vp, i64, f64, i32, vp]
        L.oracle_case_rewards.restype = None
        L.oracle_reward.argtypes = [vp, vp, i64, vp, i64, vp, i32, i64, vp, i64, f64,
                                    ctypes.c_int, u32, ctypes.c_int, ctypes.c_int, vp, vp]
        L.oracle_reward.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _prep(nodes, offsets, consts, X, y=None):
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    consts = np.ascontiguousarray(consts, dtype=np.float32)
    if consts.size == 0:
        consts = np.zeros(1, np.float32)[:0]
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim == 1:
        X = X.reshape(1, -1)
    if y is not None:
        y = np.ascontiguousarray(y, dtype=np.float32)
    return nodes, offsets, consts, X, y


def validate(nodes, offsets, n_consts, n_vars, allowed_mask=MASK_BENCH):
    """Per-program (status, max_depth)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    P = offsets.size - 1
    status = np.empty(P, np.int32)
    maxd = np.empty(P, np.int32)
    lib().oracle_validate(_ptr(nodes), _ptr(offsets), P, int(n_consts), int(n_vars),
                          allowed_mask, _ptr(status), _ptr(maxd))
    return status, maxd


def fitness(nodes, offsets, consts, X, y, tax=0.0, allowed_mask=MASK_BENCH,
            mode=M64, n_threads=0, return_threads=False):
    """Fitness per program: (F, mse, status).

    X is variable major, shape (n_vars, n_cases) or (n_vars, ld) with
    ld >= n_cases = len(y).  Invalid programs: status != 0 and F = NaN.
    """
    nodes, offsets, consts, X, y = _prep(nodes, offsets, consts, X, y)
    P = offsets.size - 1
    n_vars, ld = X.shape
    n_cases = y.size
    assert ld >= n_cases
    F = np.empty(P, np.float64)
    mse = np.empty(P, np.float64)
    status = np.empty(P, np.int32)
    used = lib().oracle_fitness(_ptr(nodes), _ptr(offsets), P, _ptr(consts), consts.size,
                                _ptr(X), n_vars, ld, _ptr(y), n_cases, float(tax),
                                allowed_mask, mode, int(n_threads), _ptr(F), _ptr(mse),
                                _ptr(status))
    if return_threads:
        return F, mse, status, used
    return F, mse, status


def correlation(nodes, offsets, consts, X, y, max_score=1e4, allowed_mask=MASK_BENCH,
                mode=M64, n_threads=0, return_counts=False):
    """Correlation score per program (the paper's Eq. 1-2): (score, r, status),
    and with return_counts the int64 counts c1 and c2 as well.

    score = M (r^2)^2 (N - (c1 + c2)) - M (c1 - c2), r over the valid pairs
    (both output and target finite), c1 = pairs with exactly one side
    invalid, c2 = pairs with both invalid.  Higher is better.  Invalid
    programs: status != 0 and score = NaN.
    """
    nodes, offsets, consts, X, y = _prep(nodes, offsets, consts, X, y)
    P = offsets.size - 1
    n_vars, ld = X.shape
    n_cases = y.size
    assert ld >= n_cases
    score = np.empty(P, np.float64)
    r = np.empty(P, np.float64)
    status = np.empty(P, np.int32)
    c12 = np.zeros((P, 2), np.int64)
    lib().oracle_correlation(_ptr(nodes), _ptr(offsets), P, _ptr(consts), consts.size,
                             _ptr(X), n_vars, ld, _ptr(y), n_cases, float(max_score),
                             allowed_mask, mode, int(n_threads), _ptr(score), _ptr(r),
                             _ptr(c12), _ptr(status))
    if return_counts:
        return score, r, status, c12[:, 0].copy(), c12[:, 1].copy()
    return score, r, status


def reward(nodes, offsets, consts, X, y, max_score=1e4, power=1, allowed_mask=MASK_BENCH,
           mode=M64, n_threads=0):
    """Integer point-to-point reward per program (the paper's Eq. 5, StdFitFunc,
    and its Square/Cube/Hyper variants for power 2, 3, 8), summed over the
    cases: (total, status).  Higher is better; invalid programs get NaN."""
    if power not in (1, 2, 3, 8):
        raise ValueError("power must be 1, 2, 3 or 8")
    if not (float(max_score) == int(max_score) and abs(max_score) <= 2 ** 24):
        raise ValueError("max_score must be an integer of magnitude <= 2^24")
    nodes, offsets, consts, X, y = _prep(nodes, offsets, consts, X, y)
    P = offsets.size - 1
    n_vars, ld = X.shape
    n_cases = y.size
    assert ld >= n_cases
    total = np.empty(P, np.float64)
    status = np.empty(P, np.int32)
    lib().oracle_reward(_ptr(nodes), _ptr(offsets), P, _ptr(consts), consts.size, _ptr(X),
                        n_vars, ld, _ptr(y), n_cases, float(max_score), int(power),
                        allowed_mask, mode, int(n_threads), _ptr(total), _ptr(status))
    return total, status


def case_rewards(o, y, max_score=1e4, power=1):
    """Per-case integer rewards (int64) of outputs ``o`` against targets
    ``y`` (same shape): the rule summed by :func:`reward`."""
    if power not in (1, 2, 3, 8):
        raise ValueError("power must be 1, 2, 3 or 8")
    o = np.ascontiguousarray(o, np.float64)
    y = np.ascontiguousarray(np.broadcast_to(np.asarray(y, np.float32), o.shape))
    out = np.empty(o.shape, np.int64)
    lib().oracle_case_rewards(_ptr(o), _ptr(y), o.size, float(max_score), int(power), _ptr(out))
    return out


def program_outputs(prog, consts, X, n_cases=None, allowed_mask=MASK_BENCH, mode=M64):
    """Per-case outputs f(x_i) of one program (a 1-D node array)."""
    prog = np.ascontiguousarray(prog, dtype=np.uint32)
    _, _, consts, X, _ = _prep(prog, [0, prog.size], consts, X)
    n_vars, ld = X.shape
    n = ld if n_cases is None else n_cases
    out = np.empty(n, np.float64)
    st = lib().oracle_program_outputs(_ptr(prog), prog.size, _ptr(consts), consts.size,
                                      _ptr(X), n_vars, ld, n, allowed_mask, mode, _ptr(out))
    if st != ST_VALID:
        raise ValueError("invalid program (status %d)" % st)
    return out


def subset(nodes, offsets, idx):
    """Programs ``idx`` of a flat population as a new (nodes, offsets)."""
    idx = np.asarray(idx, dtype=np.int64)
    lens = offsets[idx + 1] - offsets[idx]
    new_off = np.zeros(idx.size + 1, np.int64)
    np.cumsum(lens, out=new_off[1:])
    parts = [nodes[offsets[i]:offsets[i + 1]] for i in idx]
    new_nodes = np.concatenate(parts) if parts else np.zeros(0, np.uint32)
    return new_nodes.astype(np.uint32), new_off
