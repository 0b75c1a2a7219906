"""The oracle against the paper's load and overload observations (CPU only).

* App. C, per-block load figure: three choices give a lower mean load and a
  narrower spread than two, two than one, for each cost at k = 7 and 14;
* Section 2.1 / Section 4.1: an overloaded one-choice filter matches the
  exact occupancy law at every overload factor, and a 10% overload stays
  below twice the FPR with or without choices.
"""

import math

import numpy as np
import pytest

import oracle
import workload
from oracle import closed_form as cf


def moments(h):
    h = np.asarray(h, dtype=np.float64)
    j = np.arange(len(h))
    mean = (h * j).sum() / h.sum()
    return mean, math.sqrt((h * (j - mean) ** 2).sum() / h.sum())


@pytest.mark.parametrize("k", [7, 14])
def test_more_choices_lower_and_balance_the_load(k):
    n = 1 << 16
    M = math.ceil(n * k / math.log(2) / 512)
    keys = workload.positive_keys(3, n)
    for kind in (oracle.COST_MIX, oracle.COST_LA, oracle.COST_EXP):
        st = []
        for c in (1, 2, 3):
            f = oracle.OracleFilter(M, c, k, kind if c > 1 else oracle.COST_NONE, None, seed=3)
            f.insert(keys)
            h = f.block_loads()
            assert h.sum() == M
            # total load is the popcount of the filter
            assert int((h * np.arange(513, dtype=np.uint64)).sum()) == sum(bin(int(w)).count("1") for w in f.words)
            st.append(moments(h))
        (m1, s1), (m2, s2), (m3, s3) = st
        assert m3 < m2 < m1 and s3 < s2 < s1, (k, kind, st)


def test_overloaded_blocked_filter_matches_occupancy_law():
    n, k = 1 << 18, 10
    M = math.ceil(n * k / math.log(2) / 512)
    neg = workload.negative_keys(9, 4 * n, 1 << 19)
    for gamma in (1.0, 1.1, 1.5):
        f = oracle.OracleFilter(M, 1, k, oracle.COST_NONE, None, seed=9)
        m = int(gamma * n)
        f.insert(workload.positive_keys(9, m))
        assert f.conditional_fpr(neg) == pytest.approx(cf.blocked_fpr(m, M, k), rel=0.04)


def test_ten_percent_overload_costs_less_than_twice_the_fpr():
    """Section 2.1 gives 1.912 for a standard Bloom filter at k = 10."""
    n, k = 1 << 18, 10
    M = math.ceil(n * k / math.log(2) / 512)
    neg = workload.negative_keys(9, 4 * n, 1 << 19)
    for c, kind in ((1, oracle.COST_NONE), (2, oracle.COST_EXP), (3, oracle.COST_EXP)):
        fpr = []
        for gamma in (1.0, 1.1):
            f = oracle.OracleFilter(M, c, k, kind, None, seed=9)
            f.insert(workload.positive_keys(9, int(gamma * n)))
            fpr.append(f.conditional_fpr(neg))
        assert 1.5 < fpr[1] / fpr[0] < 2.2
