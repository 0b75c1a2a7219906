"""Analytic formulas of the paper, used as pins for the oracle.

TEST INFRASTRUCTURE ONLY.

* ``bloom_p0`` / ``bloom_eps``: Section 2.1, eqs. bloom:p0 and bloom:eps.
* ``max_load``: the bound behind Fig. 3A (largest per-block popcount j
  with local FPR (j/512)^k <= 2^-k / c).
* ``birthday``: Fig. 3B, probability that k uniform addresses in [512]
  are not all distinct.
* ``blocked_fpr``: exact false-positive rate of a Blocked Bloom filter
  (one choice, Section 2.2) under ideal hashing. A block that received i
  keys holds the union of i*k uniform throws into 512 bits; a negative key
  hits it with probability (P/512)^k where P is that union's size. The
  number of keys per block is Binomial(n, 1/M). The law of P after T throws
  follows from the occupancy recursion
      Pr[P_{T+1} = p] = Pr[P_T = p] p/512 + Pr[P_T = p-1] (512-p+1)/512.
* ``blocked_overhead``: the space overhead factor C(k) of a Blocked Bloom
  filter at FPR 2^-k (Fig. 1's table column), i.e. bits per key divided by k.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import optimize, stats

BITS = 512


def bloom_p0(n: float, k: int, m: float) -> float:
    """Fraction of unset bits after n*k uniform throws into m bits (eq. bloom:p0)."""
    return (1.0 - 1.0 / m) ** (n * k)


def bloom_eps(gamma: float, k: int) -> float:
    """FPR of a standard Bloom filter overloaded by gamma (eq. bloom:eps)."""
    return (1.0 - 2.0 ** (-gamma)) ** k


def max_load(c: int, k: int) -> float:
    """Largest j with (j/512)^k <= 2^-k / c, i.e. 256 * c^(-1/k) (Fig. 3A)."""
    return 256.0 * c ** (-1.0 / k)


def birthday(k: int) -> float:
    """Pr[|F(x)| < k] for k independent uniform addresses in [512] (Fig. 3B)."""
    p = 1.0
    for i in range(k):
        p *= 1.0 - i / BITS
    return 1.0 - p


def occupancy_moments(max_keys: int, k: int) -> np.ndarray:
    """g[i] = E[(P/512)^k] for a block holding the masks of i keys (i*k throws)."""
    dist = np.zeros(BITS + 1)
    dist[0] = 1.0
    p = np.arange(BITS + 1, dtype=np.float64)
    frac_k = (p / BITS) ** k
    stay = p / BITS
    move = (BITS - p) / BITS  # probability that a throw lands on a new bit given p set
    g = np.empty(max_keys + 1)
    g[0] = float(dist @ frac_k)
    for i in range(1, max_keys + 1):
        for _ in range(k):
            new = dist * stay
            new[1:] += dist[:-1] * move[:-1]
            dist = new
        g[i] = float(dist @ frac_k)
    return g


def occupancy_moments_distinct(max_keys: int, k: int) -> np.ndarray:
    """As occupancy_moments, for keys that set k distinct uniform addresses
    (App. B): with P bits set, a key adds a ~ Hypergeometric(512, 512-P, k)
    new bits; a negative key hits with probability C(P, k) / C(512, k)."""
    from scipy import special

    p = np.arange(BITS + 1)
    hit = special.comb(p, k, exact=False) / special.comb(BITS, k, exact=False)
    # transition T[P, P + a] = C(512-P, a) C(P, k-a) / C(512, k)
    T = np.zeros((BITS + 1, BITS + 1))
    for P in range(BITS + 1):
        for a in range(0, k + 1):
            if P + a <= BITS:
                T[P, P + a] = stats.hypergeom.pmf(a, BITS, BITS - P, k)
    dist = np.zeros(BITS + 1)
    dist[0] = 1.0
    g = np.empty(max_keys + 1)
    g[0] = float(dist @ hit)
    for i in range(1, max_keys + 1):
        dist = dist @ T
        g[i] = float(dist @ hit)
    return g


def blocked_fpr_distinct(n: int, M: int, k: int) -> float:
    """Exact FPR of a one-choice Blocked Bloom filter with distinct bits."""
    lam = n / M
    imax = int(lam + 12.0 * math.sqrt(lam + 1.0) + 20)
    g = occupancy_moments_distinct(imax, k)
    w = stats.binom.pmf(np.arange(imax + 1), n, 1.0 / M)
    return float(w @ g)


def blocked_fpr(n: int, M: int, k: int) -> float:
    """Exact FPR of a one-choice Blocked Bloom filter with n keys in M blocks."""
    lam = n / M
    imax = int(lam + 12.0 * math.sqrt(lam + 1.0) + 20)
    g = occupancy_moments(imax, k)
    w = stats.binom.pmf(np.arange(imax + 1), n, 1.0 / M)
    return float(w @ g)


def blocked_fpr_relative(rel_size: float, k: int, n: int = 10**9) -> float:
    """Blocked FPR when the filter has rel_size times the standard Bloom size
    m = n k / ln 2 (the x-axis of Fig. 4), with n large."""
    M = rel_size * n * k / math.log(2) / BITS
    # Poisson limit of Binomial(n, 1/M) for n large.
    lam = n / M
    imax = int(lam + 12.0 * math.sqrt(lam + 1.0) + 20)
    g = occupancy_moments(imax, k)
    w = stats.poisson.pmf(np.arange(imax + 1), lam)
    return float(w @ g)


def blocked_required_size(k: int) -> float:
    """Relative size (vs. standard Bloom) at which the blocked FPR is 2^-k."""
    target = 2.0 ** (-k)
    return float(optimize.brentq(lambda r: blocked_fpr_relative(r, k) - target, 0.8, 3.0, xtol=1e-6))


def blocked_overhead(k: int) -> float:
    """Overhead factor C(k) = required bits per key / k (Fig. 1 table)."""
    return blocked_required_size(k) / math.log(2)
