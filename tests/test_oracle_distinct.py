"""Pins for the distinct bit selection strategy (Section 3.3, App. B).

CPU only. The oracle follows the paper's procedure (raise the i-th raw value
past every earlier address at or below it, keeping the addresses sorted).
It is pinned by the worked example of App. B, by the paper's own reading of
the procedure (the i-th raw value picks that element of the addresses still
free, restated with a Python list), by the properties a uniform k-subset of
[512] has, and by an exact false-positive rate derived from the
hypergeometric law of new bits.
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


def free_list(raw):
    free = list(range(512))
    return sorted(free.pop(r) for r in raw)


def test_worked_example(paper_values):
    """App. B figure: k = 5, x = 8, f_1 = 316, then f_2 = 27 stays 27 since
    it lies below the occupied 316; values at or above 316 move up by one."""
    e = paper_values["distinct_bits_example"]
    assert oracle.distinct_positions([e["f1"], e["f2_raw"]]) == e["F_after_two"]
    assert oracle.distinct_positions([316, 316]) == [316, 317]
    assert oracle.distinct_positions([316, 315]) == [315, 316]
    assert oracle.distinct_positions([316, 510]) == [316, 511]
    # a third value in [510] with F = {27, 316}: 26 stays, 27 -> 28,
    # 314 -> 315, 315 -> 316 -> 317, 509 -> 511
    for raw3, want in ((26, 26), (27, 28), (314, 315), (315, 317), (509, 511)):
        got = oracle.distinct_positions([316, 27, raw3])
        assert got == sorted([27, 316, want])


def test_extreme_raw_values():
    for k in (1, 7, 16, 32):
        assert oracle.distinct_positions([0] * k) == list(range(k))
        assert oracle.distinct_positions([511 - i for i in range(k)]) == list(range(512 - k, 512))


@pytest.mark.parametrize("k", [1, 2, 3, 8, 14, 20, 32])
def test_procedure_equals_free_list(k):
    rnd = random.Random(k)
    for _ in range(3000):
        raw = [rnd.randrange(512 - i) for i in range(k)]
        assert oracle.distinct_positions(raw) == free_list(raw)


@pytest.mark.parametrize("k", [1, 5, 14, 32])
def test_mask_equals_set_restatement(k):
    am = workload.draw_multipliers(k + 40, k)
    for x in workload.positive_keys(k, 2000):
        m = oracle.mask(am, int(x), distinct=True)
        F = brute.bit_set_distinct(am, int(x))
        assert len(F) == k
        want = [sum(1 << (f - 64 * w) for f in F if f // 64 == w) for w in range(8)]
        assert [int(v) for v in m] == want


def test_marginals_and_gaps_are_those_of_a_uniform_subset():
    """A uniform k-subset puts each address in F with probability k/512, and
    for k = 2 the gap d = |f - f'| has Pr[d] = (512 - d) / C(512, 2)."""
    k = 8
    am = workload.draw_multipliers(3, k)
    keys = workload.positive_keys(3, 1 << 16)
    counts = np.zeros(512)
    for x in keys:
        m = oracle.mask(am, int(x), distinct=True)
        bits = np.unpackbits(m.view(np.uint8), bitorder="little")
        counts += bits
    assert counts.sum() == k * len(keys)
    assert stats.chisquare(counts).pvalue > 1e-3

    am2 = workload.draw_multipliers(4, 2)
    gaps = np.zeros(512)
    for x in workload.positive_keys(4, 1 << 17):
        F = sorted(brute.bit_set_distinct(am2, int(x)))
        gaps[F[1] - F[0]] += 1
    d = np.arange(1, 512)
    expect = (512 - d) / math.comb(512, 2) * gaps.sum()
    assert gaps[0] == 0
    assert stats.chisquare(gaps[1:], expect).pvalue > 1e-3


@pytest.mark.parametrize("M", [1, 3, 8])
def test_filter_equals_set_restatement(M):
    rnd = random.Random(100 + M)
    for c, kind in ((1, "none"), (2, "exp"), (3, "mix"), (2, "la")):
        for k in (3, 9, 17):
            bm = workload.draw_multipliers(rnd.getrandbits(32), c, coprime_to=M)
            am = workload.draw_multipliers(rnd.getrandbits(32), k)
            kid = oracle.COST_NAMES[kind]
            par = oracle.default_param(kid, k) if c > 1 else 0.0
            o = oracle.OracleFilter(M, c, k, kid, par, bm, am, distinct=True)
            b = brute.BruteFilter(M, c, k, kind, par, bm, am, distinct=True)
            keys = [int(v) for v in workload.positive_keys(rnd.getrandbits(32), 40)]
            keys += keys[:4]
            for x in keys:
                assert o.insert_one(x) == b.insert(x)
            assert [int(v) for v in o.words] == b.words()
            probe = [int(v) for v in workload.positive_keys(rnd.getrandbits(32), 300)]
            assert list(o.query(probe)) == [b.query(x) for x in probe]


def test_default_bit_multipliers_coprime_to_shrinking_moduli():
    _, am = oracle.derive_multipliers(9, 1 << 12, 2, 32, distinct=True)
    for i, a in enumerate(am):
        assert a & 1 and a >= 1 << 32 and math.gcd(a, 512 - i) == 1


def test_closed_form_against_simulation():
    """The hypergeometric occupancy chain against blocks filled with uniform
    k-subsets drawn by numpy."""
    k, i = 10, 20
    g = cf.occupancy_moments_distinct(i, k)[i]
    rng = np.random.default_rng(1)
    trials = 12000
    # each row of argsort over random keys is a uniform permutation; its
    # first k entries are a uniform k-subset
    P = np.zeros(trials, dtype=np.int64)
    for t in range(trials):
        sub = np.argsort(rng.random((i, 512)), axis=1)[:, :k]
        P[t] = len(np.unique(sub))
    vals = [math.comb(int(p), k) / math.comb(512, k) for p in P]
    assert np.mean(vals) == pytest.approx(g, rel=0.03)


def test_one_choice_fpr_matches_exact_closed_form():
    """A one-choice filter with distinct bits: the oracle's conditional FPR
    against the exact rate, and below the rate with random bits (Section 3.3:
    collisions make random selection query fewer bits)."""
    n, k = 1 << 18, 14
    M = math.ceil(n * k / math.log(2) / 512)
    bm = workload.draw_multipliers(5, 1, coprime_to=M)
    am = workload.draw_multipliers(6, k)
    keys = workload.positive_keys(5, n)
    neg = workload.negative_keys(5, n, 1 << 19)
    f = oracle.OracleFilter(M, 1, k, oracle.COST_NONE, 0.0, bm, am, distinct=True)
    f.insert(keys)
    exact = cf.blocked_fpr_distinct(n, M, k)
    assert f.conditional_fpr(neg) == pytest.approx(exact, rel=0.03)
    assert exact < cf.blocked_fpr(n, M, k)
    r = oracle.OracleFilter(M, 1, k, oracle.COST_NONE, 0.0, bm, am)
    r.insert(keys)
    assert f.conditional_fpr(neg) < r.conditional_fpr(neg)


def test_distinct_beats_random_with_choices():
    """App. D: for every cost, k and number of choices, distinct selection
    gives a smaller FPR than random selection."""
    n = 1 << 18
    neg = workload.negative_keys(7, n, 1 << 19)
    for k, c, kind in ((14, 3, oracle.COST_EXP), (10, 2, oracle.COST_MIX), (17, 2, oracle.COST_LA)):
        M = math.ceil(n * k / math.log(2) / 512)
        out = []
        for distinct in (False, True):
            f = oracle.OracleFilter(M, c, k, kind, None, seed=7, distinct=distinct)
            f.insert(workload.positive_keys(7, n))
            out.append(f.conditional_fpr(neg))
        assert out[1] < out[0]
