"""Parity gate between a device result and the fp64 oracle.

TEST INFRASTRUCTURE ONLY.

Used for the three fitness functions: the MSE fitness, the correlation
score of Eq. 1-2 (``max_score`` given) and the integer reward of Eq. 5
(``max_score`` and ``reward_power`` given).

A finite program passes when |F_dev - F_64| <= 1e-4 |F_64| + 1e-12 (the
relative tolerance of the fitness requirement, plus an absolute floor for
closed-form zeros).  Classification must be identical, and it has three
values: NaN only for a structurally invalid program (status != 0; a valid
program that comes out NaN on either side is a failure), +inf for the worst
fitness of a valid program, and finite.  A program that fails the value or
class test is examined further with the oracle's fp32-emulating modes; it
is excused only when the arithmetic itself explains it:

  * fp32 ill-conditioned: the correctly rounded fp32 evaluation (M32E)
    differs from M64 by more than 1e-5 relative, and the device result
    matches M32E within the tolerance;
  * chaotic: moving every sin/cos/exp/log/sqrt result one fp32 ulp
    (M32E_UP / M32E_DN), or by seeded pseudo-random amounts within +-2 ulps
    (M32E_RAND; the accuracy class of fp32 elementary-function code),
    changes F by more than the tolerance, or changes its class -- and the
    device value lies in the envelope of those runs: the hull of the M64,
    M32E, M32E_UP/DN and M32E_RAND results, widened on each side by its own
    width and by 4 fp32 ulps of its largest end (the rule the reward's
    output window applies per case);
  * certified class flip: the device class differs from M64's but equals
    M32E's (an fp32 overflow-range or threshold flip) or that of a
    perturbed run; a finite device value must then also lie in the
    envelope of the finite results;
  * output window (MSE and correlation): per case, the hull of the oracle's
    outputs in M64, M32E, M32E_UP/DN and the M32E_RAND runs, widened on
    each side by its own width and by 4 fp32 ulps (the same window as the
    reward's below), with every run agreeing on which outputs are finite.
    The device value must lie within what outputs anywhere in those
    windows can give: for the MSE exactly, |dF| <= (1/n) sum(2|f_i - y_i|
    w_i + w_i^2) with w_i the window's reach from the M64 output f_i; for
    the correlation score to first order in r, |dr| <= 2 sum |dr/df_i| w_i
    (the factor 2 covers the second-order terms), the correlation term
    staying within [0, M n_valid] and moving by at most
    M n_valid ((|r| + |dr|)^4 - r^4) (|r| + |dr| capped at 1); the relative
    tolerance is added on top.

The integer reward sums per-case decisions that amplify an output error
by M before rounding, so a suspicious reward is judged on the outputs
instead:

  * output window: per case, the hull of the oracle's outputs in M64, M32E,
    M32E_UP, M32E_DN and the M32E_RAND runs, widened on each side by its
    own width and by 4 fp32 ulps; the reward is piecewise monotone in the
    output (breakpoints at 0 and +-|y|), so its least and greatest value
    over the window are found among the window's ends and those
    breakpoints (the invalid-pair value joins when a candidate is not
    finite).  The device total must lie between the sums of the per-case
    least and greatest values.

Everything else is a failure.  Counts of each category are reported.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import (M32E, M32E_DN, M32E_RAND, M32E_UP, M64, case_rewards, correlation, fitness,
               program_outputs, reward, subset)

N_RANDOM = 4        # seeded random-perturbation runs per suspicious program

REL = 1e-4
ABS = 1e-12


@dataclass
class GateReport:
    n: int = 0
    n_invalid_programs: int = 0
    n_pass: int = 0
    n_ill_conditioned: int = 0
    n_chaotic: int = 0
    n_class_flip_certified: int = 0
    n_output_window: int = 0          # reward: within the output-window bounds
    n_fail: int = 0
    max_rel_err: float = 0.0          # over passing finite programs
    median_rel_err: float = 0.0
    p99_rel_err: float = 0.0
    failures: list = field(default_factory=list)

    def ok(self):
        return self.n_fail == 0

    def summary(self):
        s = ("n=%d pass=%d ill=%d chaotic=%d flip=%d fail=%d invalid=%d "
             "rel_err median=%.2g p99=%.2g max=%.3g"
             % (self.n, self.n_pass, self.n_ill_conditioned, self.n_chaotic,
                self.n_class_flip_certified, self.n_fail, self.n_invalid_programs,
                self.median_rel_err, self.p99_rel_err, self.max_rel_err))
        if self.n_output_window:
            s += " window=%d" % self.n_output_window
        return s


def window_bounds(O, y, max_score, power):
    """Per-case reward bounds over output windows.  O: [k, n] candidate
    outputs (fp64; non-finite allowed), y: [n] fp32 targets.  Returns
    (rmin, rmax, a, b): the least and greatest reward per case over the
    fp32 values in [a, b], the hull of the finite candidates widened by its
    width and 4 fp32 ulps on each side, joined with the invalid-pair value
    where a candidate is not finite."""
    y = np.ascontiguousarray(y, np.float32)
    n = y.size
    with np.errstate(over="ignore", invalid="ignore"):
        fin = np.isfinite(O) & np.isfinite(O.astype(np.float32))
    any_bad = (~fin).any(axis=0)
    all_bad = (~fin).all(axis=0)
    lo = np.where(fin, O, np.inf).min(axis=0)
    hi = np.where(fin, O, -np.inf).max(axis=0)
    lo = np.where(all_bad, 0.0, lo)
    hi = np.where(all_bad, 0.0, hi)
    width = hi - lo

    def ulp(v):
        v32 = np.minimum(np.abs(v), np.finfo(np.float32).max).astype(np.float32)
        return np.spacing(v32).astype(np.float64)

    a = lo - width - 4.0 * ulp(lo)
    b = hi + width + 4.0 * ulp(hi)
    ay = np.abs(y.astype(np.float64))
    ay = np.where(np.isnan(ay), 0.0, ay)          # a NaN target has no breakpoint
    tiny = float(np.finfo(np.float32).smallest_subnormal)
    zero = np.zeros(n)
    # window ends and the breakpoints of the piecewise-monotone reward
    cands = np.stack([np.clip(c, a, b) for c in (a, b, zero, ay, -ay, zero + tiny,
                                                 zero - tiny)])
    R = case_rewards(cands, np.broadcast_to(y, cands.shape), max_score, power)
    rmin, rmax = R.min(axis=0), R.max(axis=0)
    inv = case_rewards(np.full(n, np.nan), y, max_score, power)
    rmin = np.where(all_bad, inv, np.where(any_bad, np.minimum(rmin, inv), rmin))
    rmax = np.where(all_bad, inv, np.where(any_bad, np.maximum(rmax, inv), rmax))
    return rmin, rmax, a, b


def reward_window(prog, consts, X, y, max_score, power, allowed_mask):
    """Least and greatest integer reward of one program over the per-case
    output windows described in the module docstring: (lo, hi)."""
    y = np.ascontiguousarray(y, np.float32)
    modes = [M64, M32E, M32E_UP, M32E_DN] + [M32E_RAND + s for s in range(N_RANDOM)]
    O = np.stack([program_outputs(prog, consts, X, y.size, allowed_mask, m) for m in modes])
    rmin, rmax, _, _ = window_bounds(O, y, max_score, power)
    return int(rmin.sum()), int(rmax.sum())


def check(F_dev, nodes, offsets, consts, X, y, tax, allowed_mask, F64=None,
          status=None, n_threads=0, max_failures=20, max_score=None, reward_power=None):
    """Gate F_dev (float64[P]) against the oracle.  Returns a GateReport.

    With ``max_score`` set, F is the correlation score of Eq. 1-2 with that
    M (``tax`` unused): the relative tolerance (and the reported relative
    error) is taken on the reference's correlation term M r^4 n, and the
    invalid-pair term must agree exactly.  An absolute floor of 1e-9 M N (a
    change of 1e-9 in r^4) applies only where r^4 is about zero: where the
    correlation term itself is below the floor; everywhere else a mismatch
    beyond the relative tolerance must be certified.

    With ``reward_power`` also set, F is the integer reward of Eq. 5 (power
    1, 2, 3 or 8) summed over the cases; the relative tolerance is taken on
    |F| + 0.01 M N (rounding flips of single cases are expected between an
    fp32 and an fp64 evaluation)."""
    F_dev = np.asarray(F_dev, np.float64)
    corr = max_score is not None and reward_power is None
    if max_score is None:
        def score(nd, of, mode):
            F, _, st = fitness(nd, of, consts, X, y, tax, allowed_mask, mode, n_threads)
            return F, st, np.abs(F)
    elif reward_power is not None:
        spread = 1e-2 * float(max_score) * float(np.asarray(y).size)

        def score(nd, of, mode):
            F, st = reward(nd, of, consts, X, y, max_score, reward_power, allowed_mask, mode,
                           n_threads)
            return F, st, np.abs(F) + spread
    else:
        # the relative tolerance applies to the correlation term M r^4 n of
        # the reference; the invalid-pair term M (c1 - c2) is a multiple of
        # M and must agree exactly (a count difference moves the score by M)
        N = float(np.asarray(y).size)

        def score(nd, of, mode):
            F, r, st, c1, c2 = correlation(nd, of, consts, X, y, max_score, allowed_mask,
                                           mode, n_threads, return_counts=True)
            return F, st, float(max_score) * r ** 4 * (N - c1 - c2)

    if corr:
        MN = abs(float(max_score)) * float(np.asarray(y).size)

        def floor(T):
            # the absolute floor only where r^4 is about zero
            return np.where(np.abs(T) < 1e-9 * MN, 1e-9 * MN, ABS)
    else:
        def floor(T):
            return ABS

    def close(a, b, scale, rel=REL):
        with np.errstate(invalid="ignore"):          # inf - inf: not close
            return np.abs(a - b) <= rel * scale + floor(scale)

    if F64 is None:
        F64, status, T64 = score(nodes, offsets, M64)
    else:
        T64 = np.abs(F64)
    rep = GateReport(n=F_dev.size)
    valid = status == 0
    rep.n_invalid_programs = int(np.sum(~valid))
    bad_invalid = np.nonzero(~valid & ~np.isnan(F_dev))[0]
    for p in bad_invalid[:max_failures]:
        rep.failures.append((int(p), "invalid program not NaN", F_dev[p], F64[p]))
    rep.n_fail += bad_invalid.size
    # NaN marks a structurally invalid program only: a valid program is
    # finite or +inf on both sides
    if np.any(valid & np.isnan(F64)):
        raise AssertionError("oracle returned NaN for a valid program")
    nan_valid = np.nonzero(valid & np.isnan(F_dev))[0]
    for p in nan_valid[:max(0, max_failures - len(rep.failures))]:
        rep.failures.append((int(p), "valid program NaN", F_dev[p], F64[p]))
    rep.n_fail += nan_valid.size

    fin64 = np.isfinite(F64)
    find = np.isfinite(F_dev)
    same_class = (fin64 == find) & (fin64 | (F_dev == F64))
    good = valid & ~np.isnan(F_dev) & same_class & (~fin64 | close(F_dev, F64, T64))
    rep.n_pass = int(np.sum(good))
    # error statistics over programs well above the absolute floor (for the
    # correlation score: r^4 of at least 1e-6)
    both = valid & fin64 & find & good
    both &= (T64 >= 1e-6 * MN) if corr else (T64 > 1e3 * ABS)
    if both.any():
        rel = np.abs(F_dev[both] - F64[both]) / np.maximum(T64[both], 1e-300)
        rep.max_rel_err = float(rel.max())
        rep.median_rel_err = float(np.median(rel))
        rep.p99_rel_err = float(np.quantile(rel, 0.99))

    sus = np.nonzero(valid & ~good & ~np.isnan(F_dev))[0]
    if sus.size and reward_power is not None:
        nodes_a = np.asarray(nodes, np.uint32)
        offs_a = np.asarray(offsets, np.int64)
        for p in sus:
            lo, hi = reward_window(nodes_a[offs_a[p]:offs_a[p + 1]], consts, X, y, max_score,
                                   reward_power, allowed_mask)
            if lo <= F_dev[p] <= hi:
                rep.n_output_window += 1
                continue
            rep.n_fail += 1
            if len(rep.failures) < max_failures:
                rep.failures.append((int(p), "outside output window", F_dev[p], F64[p], lo, hi))
        return rep
    if sus.size:
        nodes_a = np.asarray(nodes, np.uint32)
        offs_a = np.asarray(offsets, np.int64)
        sn, so = subset(nodes_a, offs_a, sus)
        F32, _, T32 = score(sn, so, M32E)
        pert = [score(sn, so, m)[0]
                for m in [M32E_UP, M32E_DN] + [M32E_RAND + s for s in range(N_RANDOM)]]
        pert = np.stack(pert)
        for i, p in enumerate(sus):
            fd, f64, f32 = F_dev[p], F64[p], F32[i]
            runs = np.concatenate([[f64, f32], pert[:, i]])
            if np.isfinite(fd) != np.isfinite(f64) or (not np.isfinite(fd) and fd != f64):
                flip = "class"
                if np.isfinite(f32) == np.isfinite(fd) and (np.isfinite(fd) or fd == f32):
                    flip = "flip"
                elif np.any((np.isfinite(pert[:, i]) == np.isfinite(fd))
                            & (np.isfinite(fd) | (pert[:, i] == fd))):
                    flip = "chaotic"
                if flip != "class" and np.isfinite(fd) and not in_envelope(fd, runs):
                    flip = "class (outside envelope)"
                if flip == "flip":
                    rep.n_class_flip_certified += 1
                elif flip == "chaotic":
                    rep.n_chaotic += 1
                else:
                    rep.n_fail += 1
                    if len(rep.failures) < max_failures:
                        rep.failures.append((int(p), flip, fd, f64, f32))
                continue
            # both finite, value mismatch
            t64, t32 = T64[p], T32[i]
            ill = not close(f32, f64, t64, rel=1e-5) if np.isfinite(f32) else True
            if ill and np.isfinite(f32) and close(fd, f32, t32):
                rep.n_ill_conditioned += 1
                continue
            chaotic = (not np.all(np.isfinite(pert[:, i]))
                       or not np.all(close(pert[:, i], f32, t32)))
            if chaotic and in_envelope(fd, runs):
                rep.n_chaotic += 1
                continue
            if window_excuse(fd, f64, t64, nodes_a[offs_a[p]:offs_a[p + 1]], consts, X, y,
                             allowed_mask, max_score if corr else None):
                rep.n_output_window += 1
                continue
            rep.n_fail += 1
            if len(rep.failures) < max_failures:
                rep.failures.append((int(p), "value (chaotic, outside envelope)" if chaotic
                                     else "value", fd, f64, f32))
    return rep


def output_windows(prog, consts, X, y, allowed_mask):
    """Per-case output windows of one program: (f64, lo, hi, fin) with f64
    the M64 outputs, [lo, hi] the hull of the M64, M32E, M32E_UP/DN and
    M32E_RAND outputs widened on each side by its width and 4 fp32 ulps,
    and fin the cases where every run's output is finite (None when the
    runs disagree on which outputs are finite)."""
    n = np.asarray(y).size
    modes = [M64, M32E, M32E_UP, M32E_DN] + [M32E_RAND + s for s in range(N_RANDOM)]
    O = np.stack([program_outputs(prog, consts, X, n, allowed_mask, m) for m in modes])
    with np.errstate(over="ignore", invalid="ignore"):
        fin_all = np.isfinite(O) & np.isfinite(O.astype(np.float32))
    fin = fin_all.all(axis=0)
    if not np.array_equal(fin, fin_all.any(axis=0)):
        return None
    Of = np.where(fin, O, 0.0)
    lo, hi = Of.min(axis=0), Of.max(axis=0)
    w = hi - lo

    def ulp(v):
        v32 = np.minimum(np.abs(v), np.finfo(np.float32).max).astype(np.float32)
        return np.spacing(v32).astype(np.float64)

    return O[0], lo - w - 4.0 * ulp(lo), hi + w + 4.0 * ulp(hi), fin


def window_excuse(fd, f64, t64, prog, consts, X, y, allowed_mask, max_score=None):
    """Whether the finite device value fd of one program lies within what
    outputs anywhere in its per-case output windows can give (the bounds in
    the module docstring), the relative tolerance added on top."""
    ow = output_windows(prog, consts, X, y, allowed_mask)
    if ow is None:
        return False
    f, lo, hi, fin = ow
    yy = np.asarray(y, np.float32).astype(np.float64)
    v = fin & np.isfinite(yy)                      # valid pairs
    reach = np.where(v, np.maximum(hi - f, f - lo), 0.0)
    if max_score is None:
        n = yy.size
        bound = float(np.sum(2.0 * np.abs(np.where(v, f - yy, 0.0)) * reach + reach * reach)) / n
        return abs(fd - f64) <= REL * abs(t64) + bound + ABS
    M = abs(float(max_score))
    nv = int(v.sum())
    c1 = int(np.sum(fin != np.isfinite(yy)))
    c2 = int(np.sum(~fin & ~np.isfinite(yy)))
    T_dev = fd + float(max_score) * (c1 - c2)          # the device's correlation term
    if not (-1e-6 * M * max(nv, 1) <= T_dev * np.sign(max_score) <= M * nv * (1 + 1e-6)):
        return False
    if nv < 2:
        return abs(fd - f64) <= REL * abs(t64) + ABS
    fv, yv = f[v], yy[v]
    df, dy = fv - fv.mean(), yv - yv.mean()
    sxx, syy = float(np.dot(df, df)), float(np.dot(dy, dy))
    if sxx == 0.0 or syy == 0.0:
        r, dr = 0.0, (1.0 if syy > 0.0 and np.any(reach[v] > 0.0) else 0.0)
    else:
        r = float(np.dot(df, dy)) / np.sqrt(sxx * syy)
        grad = dy / np.sqrt(sxx * syy) - r * df / sxx
        dr = 2.0 * float(np.sum(np.abs(grad) * reach[v]))
    top = min(1.0, abs(r) + dr)
    bound = M * nv * (top ** 4 - r ** 4)
    return abs(fd - f64) <= REL * abs(t64) + bound + ABS


def envelope(runs):
    """The interval of values certified by a set of oracle runs: the hull of
    the finite results, widened on each side by its own width and by 4 fp32
    ulps of its largest end (None when no run is finite)."""
    runs = np.asarray(runs, np.float64)
    fin = runs[np.isfinite(runs)]
    if fin.size == 0:
        return None
    lo, hi = float(fin.min()), float(fin.max())
    w = hi - lo
    ulp = float(np.spacing(np.float32(min(max(abs(lo), abs(hi)), np.finfo(np.float32).max))))
    return lo - w - 4.0 * ulp, hi + w + 4.0 * ulp


def in_envelope(v, runs):
    env = envelope(runs)
    return env is not None and env[0] <= v <= env[1]
