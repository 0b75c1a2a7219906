"""Pins for the sub-array layout (Section 3.4, "Parallelization").

CPU only. The filter's M blocks form T sub-arrays of S = M/T blocks; h_0
picks a key's sub-array and the block hashes h_i map into [S]. Pinned by the
set-based restatement, by the definition itself (a sub-array filter is T
independent S-block filters, each fed the keys h_0 sends to it, in order),
by uniformity of h_0, by the one-choice closed form (every block is still
uniform) and by the false-positive rate staying that of a single array.
"""

import math
import random

import numpy as np
import pytest
from scipy import stats

import oracle
import workload
from oracle import brute
from oracle import closed_form as cf


@pytest.mark.parametrize("M,T", [(4, 2), (6, 3), (6, 2), (12, 4), (64, 8), (60, 5), (7, 7)])
def test_equals_set_restatement(M, T):
    rnd = random.Random(M * 100 + T)
    S = M // T
    for c, kind in ((1, "none"), (2, "exp"), (3, "mix"), (2, "la")):
        for k in (2, 6, 11):
            bm = workload.draw_multipliers(rnd.getrandbits(32), c, coprime_to=S)
            am = workload.draw_multipliers(rnd.getrandbits(32), k)
            sm = workload.draw_multipliers(rnd.getrandbits(32), 1, coprime_to=T)[0]
            kid = oracle.COST_NAMES[kind]
            par = oracle.default_param(kid, k) if c > 1 else 0.0
            o = oracle.OracleFilter(M, c, k, kid, par, bm, am, subarrays=T, sub_mult=sm)
            b = brute.BruteFilter(M, c, k, kind, par, bm, am, subarrays=T, sub_mult=sm)
            keys = [int(v) for v in workload.positive_keys(rnd.getrandbits(32), 60)]
            keys += keys[:5]
            for x in keys:
                assert o.insert_one(x) == b.insert(x)
            assert [int(v) for v in o.words] == b.words()
            probe = [int(v) for v in workload.positive_keys(rnd.getrandbits(32), 300)]
            assert list(o.query(probe)) == [b.query(x) for x in probe]


@pytest.mark.parametrize("T,S,c,kind", [(16, 64, 2, oracle.COST_LA), (6, 50, 3, oracle.COST_EXP),
                                        (8, 32, 1, oracle.COST_NONE)])
def test_subarray_filter_is_independent_filters(T, S, c, kind):
    """Section 3.4: sub-array t holds exactly what an S-block filter holds
    after inserting, in order, the keys with h_0(x) = t."""
    M, k = T * S, 9
    bm = workload.draw_multipliers(1, c, coprime_to=S)
    am = workload.draw_multipliers(2, k)
    sm = workload.draw_multipliers(3, 1, coprime_to=T)[0]
    keys = workload.positive_keys(4, S * T * 20)
    f = oracle.OracleFilter(M, c, k, kind, None, bm, am, subarrays=T, sub_mult=sm)
    f.insert(keys)
    h0 = np.array([oracle.hash_(sm, int(x), T) for x in keys])
    neg = workload.negative_keys(4, len(keys), 4000)
    hn = np.array([oracle.hash_(sm, int(x), T) for x in neg])
    got = f.query(neg)
    for t in range(T):
        g = oracle.OracleFilter(S, c, k, kind, None, bm, am)
        g.insert(keys[h0 == t])
        assert np.array_equal(f.words[8 * S * t:8 * S * (t + 1)], g.words), t
        assert np.array_equal(got[hn == t], g.query(neg[hn == t]))


@pytest.mark.parametrize("T", [2 ** 10, 3 * 7 * 11, 1000])
def test_subarray_hash_is_uniform(T):
    sm = workload.draw_multipliers(T, 1, coprime_to=T)[0]
    keys = workload.positive_keys(T, 200 * T)
    counts = np.bincount([oracle.hash_(sm, int(x), T) for x in keys], minlength=T)
    assert stats.chisquare(counts).pvalue > 1e-3


def test_block_index_layout():
    """Candidate i of x is block h_0(x) S + h_i(x)."""
    M, T = 96, 8
    S = M // T
    for x in workload.positive_keys(5, 200):
        x = int(x)
        for a in workload.draw_multipliers(6, 3, coprime_to=S):
            want = oracle.hash_(77 | (1 << 40), x, T) * S + oracle.hash_(a, x, S)
            assert oracle.block_index(M, T, 77 | (1 << 40), a, x) == want
    assert oracle.block_index(M, 1, 0, 5 | (1 << 40), 12345) == oracle.hash_(5 | (1 << 40), 12345, M)


def test_default_sub_multiplier_follows_the_bit_multipliers():
    """R3: block multipliers (coprime to S), bit multipliers, then h_0's."""
    M, T, c, k = 3 * 4096, 3 * 64, 2, 5
    bm, am, sm = oracle.derive_multipliers(8, M, c, k, subarrays=T, with_sub=True)
    rng = workload.SplitMix64(8)
    draws = []
    while len(draws) < c + k + 1:
        a = rng.next() | 1
        mod = M // T if len(draws) < c else (512 if len(draws) < c + k else T)
        if a >= 1 << 32 and math.gcd(a, mod) == 1:
            draws.append(a)
    assert bm + am + [sm] == draws
    assert oracle.derive_multipliers(8, M, c, k, subarrays=1, with_sub=True)[2] == 0


def test_one_choice_subarray_fpr_matches_closed_form():
    """With one choice every block is still uniform over the M blocks, so
    the exact Blocked Bloom FPR (Section 2.2) holds for any T."""
    n, k = 1 << 19, 10
    S = 512
    M = math.ceil(n * k / math.log(2) / 512 / S) * S
    f = oracle.OracleFilter(M, 1, k, oracle.COST_NONE, None, seed=2, subarrays=M // S)
    f.insert(workload.positive_keys(2, n))
    neg = workload.negative_keys(2, n, 1 << 19)
    assert f.conditional_fpr(neg) == pytest.approx(cf.blocked_fpr(n, M, k), rel=0.03)


def test_choices_fpr_unchanged_by_small_subarrays():
    """16 bits per key, k = 11, two choices, LA: sub-arrays of 512 and 1024
    blocks keep the FPR of one array within 1.5% (the per-sub-array key count
    varies by about 1/sqrt(32 S))."""
    n = 1 << 20
    M = n // 32
    neg = workload.negative_keys(3, n, 1 << 20)
    fpr = {}
    for T in (1, M // 1024, M // 512):
        f = oracle.OracleFilter(M, 2, 11, oracle.COST_LA, None, seed=3, subarrays=T)
        f.insert(workload.positive_keys(3, n))
        fpr[T] = f.conditional_fpr(neg)
    for T in (M // 1024, M // 512):
        assert fpr[T] == pytest.approx(fpr[1], rel=0.015), fpr
