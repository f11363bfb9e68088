"""Seeded synthetic workloads: random postfix populations and fitness cases.

This module is plain input generation; it holds none of the scoring
arithmetic and imports nothing from the library or from the oracle, so both
sides can be fed the same arrays.

Program arrays (the library's interchange format):
    nodes   uint32[sum len]   node = op | (arg << 8)
    offsets int64[P + 1]      program p is nodes[offsets[p]:offsets[p+1]]
    consts  float32[C]        constant pool, CONST arg indexes it
    X       float32[n_vars][n_cases]  variable major
    y       float32[n_cases]

Op numbering: LOAD 0, CONST 1, ADD 2, SUB 3, MUL 4, DIV 5, SIN 6, COS 7,
EXP 8, LOG 9, SQRT 10, ABS 11; the rest of the GCL command table: DUP 12,
SWAP 13, DEL 14, SQUARE 15, SIGN 16, CUBE 17, CBRT 18, TAN 19, ARCSIN 20,
ARCCOS 21, ARCTAN 22, TANH 23, SQRT_RAW 24, POW 25, COPY 26, PASTE 27 (COPY
and PASTE carry a variable name k < 16 in the arg field).

Workload recipes (fixed for this project; the paper benchmarks on data it
does not ship, so these stand in for it):
  plain             1,000 programs, len U{3..32}, {+,-,*,/,sin,cos,exp,log},
                    3 vars, 1,024 cases, X ~ U(-1,1),
                    y = x0^2 + sin(x1) x2 + N(0, sd 0.01), tax 0
  generation        100,000 programs, len U{3..64}, set 1 + {sqrt, abs},
                    5 vars, 4,096 cases, X ~ U(-3,3), y = dense degree<=3
                    polynomial (56 monomials, coef U(-1,1)) + N(0, 0.05),
                    tax 1e-3
  uneven            1,000,000 programs, len clip(Geom(1/24), 3, 128), set 2,
                    10 vars, 16,384 cases, X ~ N(0,1), y as generation (286
                    monomials)
  precision         50,000 programs, len U{3..64}, set 2, 3 vars,
                    1,048,576 cases, X ~ U(-10,10), y = degree-3 polynomial
                    (20 monomials) scaled to max|y| = 1e4, no noise
  gcl               20,000 programs, len U{3..48}, the whole GCL command
                    table (sample_gcl_programs), 4 vars, 2,048 cases,
                    X ~ U(-1,1), y = x0^2 + sin(x1) x2 - x3/2 + N(0, 0.01),
                    tax 1e-3
  serving           64 runs, each n_vars U{1..20}, cases log-U[256, 65536],
                    X ~ N(0,1), y = <=32 random degree<=3 monomials + N(0,
                    0.05); requests of log-U[1k, 200k] programs, len
                    U{3..128}, set 2

Program sampler: length L from the workload's length law; tokens left to right with
current depth d and r tokens still to come after this one.  A class is
feasible when: leaf d+1 <= 32 and d <= r; unary d >= 1 and d-1 <= r; binary
d >= 2 and d-2 <= r.  A feasible class is picked uniformly, then an op
uniformly inside it; a leaf is a variable (uniform index) with probability
1/2, else a constant U(-5,5) rounded to fp32.  Never dead-ends, always ends
at depth 1, never exceeds depth 32.  (With no unary op in the set, the
lengths must be odd and a class is also required to leave an even number of
tokens to pair up.)
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

LOAD, CONST, ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, ABS = range(12)
(DUP, SWAP, DEL, SQUARE, SIGN, CUBE, CBRT, TAN, ASIN, ACOS, ATAN, TANH, SQRT_RAW, POW,
 COPY, PASTE) = range(12, 28)
N_OPS = 28
BINARY = (ADD, SUB, MUL, DIV)
UNARY_1 = (SIN, COS, EXP, LOG)
UNARY_2 = (SIN, COS, EXP, LOG, SQRT, ABS)
UNARY_GCL = UNARY_2 + (SQUARE, SIGN, CUBE, CBRT, TAN, ASIN, ACOS, ATAN, TANH, SQRT_RAW)
BINARY_GCL = BINARY + (POW,)
STACK_LIMIT = 32
GCL_VARS = 16


def op_mask(ops):
    m = (1 << LOAD) | (1 << CONST)
    for o in ops:
        m |= 1 << o
    return m


MASK_1 = op_mask(BINARY + UNARY_1)
MASK_2 = op_mask(BINARY + UNARY_2)
MASK_GCL = (1 << N_OPS) - 1


@dataclass
class Population:
    nodes: np.ndarray
    offsets: np.ndarray
    consts: np.ndarray

    @property
    def n_programs(self):
        return self.offsets.size - 1

    @property
    def lengths(self):
        return np.diff(self.offsets)

    def take(self, idx):
        """Programs ``idx`` as a new population (constants re-indexed)."""
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.offsets[idx + 1] - self.offsets[idx]
        off = np.zeros(idx.size + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        sel = _ranges(self.offsets[idx], lens)
        nodes = self.nodes[sel].copy()
        is_c = (nodes & 0xFF) == CONST
        old = (nodes[is_c] >> 8).astype(np.int64)
        consts = self.consts[old].copy()
        nodes[is_c] = CONST | (np.arange(old.size, dtype=np.uint32) << 8)
        return Population(nodes.astype(np.uint32), off, consts.astype(np.float32))


def _ranges(starts, lens):
    total = int(lens.sum())
    rep = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return np.arange(total, dtype=np.int64) + rep


@dataclass
class Dataset:
    X: np.ndarray          # float32 [n_vars, n_cases]
    y: np.ndarray          # float32 [n_cases]

    @property
    def n_vars(self):
        return self.X.shape[0]

    @property
    def n_cases(self):
        return self.y.size


@dataclass
class Workload:
    name: str
    pop: Population
    data: Dataset
    tax: float
    allowed_mask: int
    extra: dict = field(default_factory=dict)

    @property
    def node_evals(self):
        return int(self.pop.offsets[-1]) * int(self.data.n_cases)


# Each workload draws from its own seed stream (default entropy 1000 + id).
WORKLOAD_IDS = {"plain": 1, "generation": 2, "uneven": 3, "precision": 4, "serving": 5,
                "gcl": 6}
WORKLOADS = ("plain", "generation", "uneven", "precision", "gcl")


def _rngs(name, seed=None):
    k = WORKLOAD_IDS[name]
    ss = np.random.SeedSequence(1000 + k if seed is None else seed)
    kids = ss.spawn(5)
    return [np.random.Generator(np.random.PCG64(s)) for s in kids]


def sample_programs(rng, lengths, n_vars, unary, binary=BINARY,
                    const_lo=-5.0, const_hi=5.0, p_var=0.5):
    """Vectorised sampler (see module docstring)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    P = lengths.size
    offsets = np.zeros(P + 1, np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    nodes = np.zeros(total, np.uint32)
    is_const = np.zeros(total, bool)
    const_val = np.zeros(total, np.float32)
    depth = np.zeros(P, np.int64)
    unary = np.asarray(unary, np.uint32)
    binary = np.asarray(binary, np.uint32)
    has_unary = unary.size > 0
    if not has_unary:
        assert np.all(lengths % 2 == 1), "without unary ops lengths must be odd"
    maxL = int(lengths.max()) if P else 0
    order = np.argsort(-lengths, kind="stable")
    sorted_len = lengths[order]
    for t in range(maxL):
        n_act = int(np.searchsorted(-sorted_len, -t, side="left"))
        act = order[:n_act]
        d = depth[act]
        r = lengths[act] - t - 1
        f_leaf = (d + 1 <= STACK_LIMIT) & (d <= r)
        f_un = (d >= 1) & (d - 1 <= r) & has_unary
        f_bin = (d >= 2) & (d - 2 <= r)
        if not has_unary:
            # without depth-neutral ops the remaining tokens must pair up
            even = ((r - d) % 2) == 0
            f_leaf &= even
            f_bin &= even
        nf = f_leaf.astype(np.int64) + f_un + f_bin
        pick = np.minimum((rng.random(n_act) * nf).astype(np.int64), nf - 1)
        # pick-th feasible class in the order leaf, unary, binary
        cls = np.where(f_leaf & (pick == 0), 0,
              np.where(f_un & (pick == f_leaf.astype(np.int64)), 1, 2))
        pos = offsets[act] + t
        u_op = rng.integers(0, max(unary.size, 1), n_act)
        b_op = rng.integers(0, binary.size, n_act)
        var_leaf = rng.random(n_act) < p_var
        var_idx = rng.integers(0, n_vars, n_act)
        cval = rng.uniform(const_lo, const_hi, n_act).astype(np.float32)
        leaf = cls == 0
        if has_unary:
            nodes[pos[cls == 1]] = unary[u_op[cls == 1]]
        nodes[pos[cls == 2]] = binary[b_op[cls == 2]]
        lv = leaf & var_leaf
        nodes[pos[lv]] = LOAD | (var_idx[lv].astype(np.uint32) << 8)
        lc = leaf & ~var_leaf
        is_const[pos[lc]] = True
        const_val[pos[lc]] = cval[lc]
        depth[act] = d + np.where(cls == 0, 1, np.where(cls == 1, 0, -1))
    assert np.all(depth == 1)
    cpos = np.nonzero(is_const)[0]
    consts = const_val[cpos].copy()
    nodes[cpos] = CONST | (np.arange(cpos.size, dtype=np.uint32) << 8)
    return Population(nodes, offsets, consts)


# token classes of the GCL sampler and their weights
_GCL_CLASSES = ("leaf", "unary", "binary", "dup", "swap", "del", "copy", "paste")
_GCL_WEIGHTS = np.array([3.0, 2.0, 3.0, 0.6, 0.6, 0.4, 0.5, 1.5])


def sample_gcl_programs(rng, lengths, n_vars, const_lo=-5.0, const_hi=5.0, p_var=0.5,
                        p_pow=0.04, unary=UNARY_GCL, binary=BINARY):
    """Programs over the whole GCL command table, one token at a time.

    State: depth d, live variables l, r tokens still to come after this one.
    A class is feasible when its result keeps d + l <= 32 and can still end
    at depth 1 with every variable pasted (each live variable needs a PASTE
    and a binary op: d' - 1 + 2 l' <= r):
      leaf d+1; unary d >= 1; binary d >= 2; DUP d >= 1, d+1; SWAP d >= 2;
      DEL d >= 2, d-1; COPY d >= 1, l < 16, l+1; PASTE l >= 1, d+1, l-1.
    A feasible class is drawn with the weights above, then an op uniformly
    inside it (unary from ``unary``; POW with probability p_pow, else one of
    ``binary``); COPY takes
    the lowest free variable name, PASTE a live one uniformly.  Leaves are
    as in sample_programs.  Never dead-ends (PASTE, a binary op, a unary op
    or a leaf stays feasible), ends at depth 1 with no live variable."""
    lengths = np.asarray(lengths, dtype=np.int64)
    P = lengths.size
    offsets = np.zeros(P + 1, np.int64)
    np.cumsum(lengths, out=offsets[1:])
    nodes = np.zeros(int(offsets[-1]), np.uint32)
    consts = []
    unary = np.array(unary, np.uint32)
    nb = len(binary)
    for p in range(P):
        Lp = int(lengths[p])
        d, live = 0, []
        pos = int(offsets[p])
        u = rng.random((Lp, 5))
        for t in range(Lp):
            r = Lp - t - 1
            l = len(live)
            feas = np.array([
                d + 1 + l <= STACK_LIMIT and d + 2 * l <= r,             # leaf
                d >= 1 and d - 1 + 2 * l <= r,                            # unary
                d >= 2 and d - 2 + 2 * l <= r,                            # binary
                d >= 1 and d + 1 + l <= STACK_LIMIT and d + 2 * l <= r,   # dup
                d >= 2 and d - 1 + 2 * l <= r,                            # swap
                d >= 2 and d - 2 + 2 * l <= r,                            # del
                d >= 1 and l < GCL_VARS and d + l + 1 <= STACK_LIMIT
                and d + 1 + 2 * l <= r,                                   # copy
                l >= 1 and d + 2 * (l - 1) <= r,                          # paste
            ])
            w = _GCL_WEIGHTS * feas
            cls = _GCL_CLASSES[min(int(np.searchsorted(np.cumsum(w), u[t, 0] * w.sum(),
                                                       side="right")), 7)]
            if cls == "leaf":
                if u[t, 1] < p_var:
                    tok = LOAD | (min(int(u[t, 2] * n_vars), n_vars - 1) << 8)
                else:
                    consts.append(np.float32(const_lo + (const_hi - const_lo) * u[t, 2]))
                    tok = CONST | ((len(consts) - 1) << 8)
                d += 1
            elif cls == "unary":
                tok = int(unary[min(int(u[t, 1] * unary.size), unary.size - 1)])
            elif cls == "binary":
                tok = POW if u[t, 1] < p_pow else binary[min(int(u[t, 2] * nb), nb - 1)]
                d -= 1
            elif cls == "dup":
                tok = DUP
                d += 1
            elif cls == "swap":
                tok = SWAP
            elif cls == "del":
                tok = DEL
                d -= 1
            elif cls == "copy":
                k = min(set(range(GCL_VARS)) - set(live))
                live.append(k)
                tok = COPY | (k << 8)
            else:
                k = live.pop(min(int(u[t, 1] * l), l - 1))
                tok = PASTE | (k << 8)
                d += 1
            nodes[pos + t] = tok
        assert d == 1 and not live
    return Population(nodes, offsets, np.array(consts, np.float32))


def monomials(n_vars, degree=3):
    """All exponent tuples of total degree <= degree (constant term first)."""
    out = []
    for deg in range(degree + 1):
        for combo in itertools.combinations_with_replacement(range(n_vars), deg):
            out.append(combo)
    return out


def poly_eval(X64, terms, coefs):
    y = np.zeros(X64.shape[1], np.float64)
    for combo, c in zip(terms, coefs):
        t = np.full(X64.shape[1], c, np.float64)
        for v in combo:
            t = t * X64[v]
        y += t
    return y


def length_law(name, rng, n):
    if name == "plain":
        return rng.integers(3, 33, n)
    if name in ("generation", "precision"):
        return rng.integers(3, 65, n)
    if name == "uneven":
        return np.clip(rng.geometric(1.0 / 24.0, n), 3, 128)
    if name == "serving":
        return rng.integers(3, 129, n)
    if name == "gcl":
        return rng.integers(3, 49, n)
    raise ValueError(name)


# programs, cases, variables at full size
SIZES = {"plain": (1_000, 1_024, 3), "generation": (100_000, 4_096, 5),
         "uneven": (1_000_000, 16_384, 10), "precision": (50_000, 1_048_576, 3),
         "gcl": (20_000, 2_048, 4)}


def make_dataset(name, n_cases=None, seed=None):
    rp, rx, rpoly, rnoise, _ = _rngs(name, seed)
    _, n_default, n_vars = SIZES[name]
    n = n_default if n_cases is None else int(n_cases)
    if name == "plain":
        X = rx.uniform(-1, 1, (n_vars, n)).astype(np.float32)
        X64 = X.astype(np.float64)
        y = X64[0] ** 2 + np.sin(X64[1]) * X64[2] + rnoise.normal(0, 0.01, n)
    elif name == "generation":
        X = rx.uniform(-3, 3, (n_vars, n)).astype(np.float32)
        terms = monomials(n_vars)
        y = poly_eval(X.astype(np.float64), terms, rpoly.uniform(-1, 1, len(terms)))
        y += rnoise.normal(0, 0.05, n)
    elif name == "uneven":
        X = rx.standard_normal((n_vars, n)).astype(np.float32)
        terms = monomials(n_vars)
        y = poly_eval(X.astype(np.float64), terms, rpoly.uniform(-1, 1, len(terms)))
        y += rnoise.normal(0, 0.05, n)
    elif name == "precision":
        X = rx.uniform(-10, 10, (n_vars, n)).astype(np.float32)
        terms = monomials(n_vars)
        y = poly_eval(X.astype(np.float64), terms, rpoly.uniform(-1, 1, len(terms)))
        y *= 1e4 / np.max(np.abs(y))
    elif name == "gcl":
        X = rx.uniform(-1, 1, (n_vars, n)).astype(np.float32)
        X64 = X.astype(np.float64)
        y = X64[0] ** 2 + np.sin(X64[1]) * X64[2] - 0.5 * X64[3] + rnoise.normal(0, 0.01, n)
    else:
        raise ValueError(name)
    return Dataset(np.ascontiguousarray(X), y.astype(np.float32))


def make_workload(name, n_programs=None, n_cases=None, seed=None):
    """Workload ``name`` (one of WORKLOADS) at its full size, or with sizes
    overridden."""
    rp = _rngs(name, seed)[0]
    P_default, _, n_vars = SIZES[name]
    P = P_default if n_programs is None else int(n_programs)
    plain = name == "plain"
    if name == "gcl":
        pop = sample_gcl_programs(rp, length_law(name, rp, P), n_vars)
    else:
        pop = sample_programs(rp, length_law(name, rp, P), n_vars,
                              UNARY_1 if plain else UNARY_2)
    data = make_dataset(name, n_cases, seed)
    tax = 0.0 if plain else 1e-3
    mask = MASK_1 if plain else (MASK_GCL if name == "gcl" else MASK_2)
    return Workload(name, pop, data, tax, mask)


# ---------------------------------------------------------------- serving
@dataclass
class ServingRun:
    run_id: int
    data: Dataset


def make_serving_runs(n_runs=64, seed=None, max_cases=65536):
    """Serving datasets: one resident dataset per evolutionary run."""
    _, rx, rpoly, rnoise, _ = _rngs("serving", seed)
    runs = []
    for r in range(n_runs):
        n_vars = int(rx.integers(1, 21))
        n = int(np.exp(rx.uniform(np.log(256), np.log(max_cases + 1))))
        n = min(max(n, 256), max_cases)
        X = rx.standard_normal((n_vars, n)).astype(np.float32)
        terms = monomials(n_vars)
        n_terms = int(rpoly.integers(1, 33))
        pick = rpoly.choice(len(terms), size=min(n_terms, len(terms)), replace=False)
        coefs = rpoly.uniform(-1, 1, pick.size)
        y = poly_eval(X.astype(np.float64), [terms[i] for i in pick], coefs)
        y += rnoise.normal(0, 0.05, n)
        runs.append(ServingRun(r, Dataset(X, y.astype(np.float32))))
    return runs


def make_serving_request(rng, run, min_pop=1_000, max_pop=200_000):
    """One scoring request (a population) for ``run``."""
    P = int(np.exp(rng.uniform(np.log(min_pop), np.log(max_pop + 1))))
    P = min(max(P, min_pop), max_pop)
    return sample_programs(rng, rng.integers(3, 129, P), run.data.n_vars, UNARY_2)
