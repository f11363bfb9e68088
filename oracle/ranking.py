"""Monte-Carlo ranking (the paper's Sec. "Monte-Carlo Ranking", Table 2),
written out plainly.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product
path; it shares no code with the HIP library.

Definition (the readings are listed in the design notes):
  * sample: draw k = 0..S-1 picks individual floor(h_k * n / 2^64), where
    h_k is the k-th output of SplitMix64 (Steele, Lea, Flood 2014) started
    at the seed; draws are with replacement;
  * key(v) = v when higher is better, else -v; NaN is -inf (the worst);
  * an individual's percentile is floor(100 * c / S), c = the number of
    sampled keys strictly below its key (ties are not beaten);
  * its band is the percentile's tens (0, 10, ..., 90; 90 and above is the
    top band), and its expected number of children is Table 2's entry.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

#: Table 2: expected number of children by percentile band
CHILDREN = {90: 4.0, 80: 2.5, 70: 1.5, 60: 1.0, 50: 0.5, 40: 0.25, 30: 0.15,
            20: 0.06, 10: 0.03, 0: 0.01}


def splitmix64(state):
    """One SplitMix64 step: (new state, output)."""
    state = (state + GAMMA) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def sample_indices(n, seed, S):
    """The S sampled individuals (with replacement)."""
    out = []
    state = seed & MASK64
    for _ in range(S):
        state, h = splitmix64(state)
        out.append((h * n) >> 64)
    return out


def keys(fitness, higher_is_better):
    f = np.asarray(fitness, np.float64)
    k = f.copy() if higher_is_better else -f
    k[np.isnan(f)] = -np.inf
    return k


def mc_rank(fitness, higher_is_better, seed, S=100):
    """(band int32[n], children float32[n], sorted sample keys float64[S])."""
    fitness = np.asarray(fitness, np.float64)
    n = fitness.size
    kk = keys(fitness, higher_is_better)
    sample = np.array([kk[i] for i in sample_indices(n, seed, S)], np.float64)
    counts = np.empty(n, np.int64)
    for lo in range(0, n, 4096):
        counts[lo:lo + 4096] = (sample[None, :] < kk[lo:lo + 4096, None]).sum(axis=1)
    pct = (100 * counts) // S
    band = (np.minimum(pct // 10, 9) * 10).astype(np.int32)
    children = np.array([CHILDREN[int(b)] for b in band], np.float32)
    return band, children, np.sort(sample)
