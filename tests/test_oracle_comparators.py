"""Pins of the oracle's test-side functions: the envelope that bounds a
racing insert, the per-block load histogram, the mixed cost's sigma, and the
conditional false-positive estimate for two or more choices.

CPU only. Each pin compares the oracle with something other than itself:
the set-based restatement (``oracle/brute.py``), the method's reductions
(M = 1, c = 1), exact rational arithmetic, or brute-force enumeration of all
bit-address pairs.
"""

import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workload
from oracle import brute

GOLDEN = (1 + math.sqrt(5)) / 2


def _popcount(words: np.ndarray) -> int:
    return int(np.bitwise_count(np.asarray(words, dtype=np.uint64)).sum())


def _random_words(rng: np.random.Generator, n_words: int, density: float) -> np.ndarray:
    """Words whose bits are set independently with probability `density`."""
    bits = rng.random((n_words, 64)) < density
    weights = np.left_shift(np.uint64(1), np.arange(64, dtype=np.uint64))
    return np.ascontiguousarray((bits.astype(np.uint64) * weights).sum(axis=1, dtype=np.uint64))


# ------------------------------------------------------------- envelope
# Sections 3.1 and 3.2: a racing insert places each key's F(x) in one of its
# candidates (or finds it present), so any filter it can produce lies inside
# the OR of every key's mask into every candidate.

def test_envelope_with_one_choice_is_the_filter():
    """c = 1: each key has a single candidate, so the envelope is exactly the
    one-choice filter (Section 2.2), built in any key order."""
    for M, k, seed in ((97, 9, 3), (1 << 10, 14, 4), (6, 5, 5)):
        keys = workload.positive_keys(seed, 3000)
        f = oracle.OracleFilter(M, 1, k, oracle.COST_NONE, None, seed=seed)
        f.insert(np.random.default_rng(seed).permutation(keys))
        assert np.array_equal(f.envelope(keys), f.words)


@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_envelope_of_one_block_is_or_of_masks(c):
    """M = 1: every candidate is block 0, so the envelope is the OR of all
    masks, a 512-bit standard Bloom filter (Section 2.1)."""
    k = 7
    kind = oracle.COST_NONE if c == 1 else oracle.COST_EXP
    f = oracle.OracleFilter(1, c, k, kind, None, [(1 << 33) | 1] * c, workload.draw_multipliers(31, k))
    keys = workload.positive_keys(31, 25)
    acc = np.zeros(8, dtype=np.uint64)
    for x in keys:
        acc |= oracle.mask(f.bit_mult, int(x))
    assert np.array_equal(f.envelope(keys), acc)
    assert 0 < _popcount(acc) < 512


@pytest.mark.parametrize("M", [2, 3, 4, 5, 6, 8, 12, 64])
def test_envelope_equals_set_restatement(M):
    """c >= 2: word for word equal to the set-based envelope, for every hash
    case of M, both bit selections and a sub-array layout."""
    rnd = random.Random(100 + M)
    for c in (2, 3, 4):
        for distinct in (False, True):
            for T in (1, 2) if M % 2 == 0 else (1,):
                k = rnd.choice([3, 6, 11])
                S = M // T
                bm = workload.draw_multipliers(rnd.getrandbits(32), c, coprime_to=S)
                am = (workload.draw_multipliers(rnd.getrandbits(32), k) if not distinct else
                      oracle.derive_multipliers(rnd.getrandbits(32), M, c, k, True)[1])
                sm = workload.draw_multipliers(rnd.getrandbits(32), 1, coprime_to=T)[0] if T > 1 else 0
                o = oracle.OracleFilter(M, c, k, oracle.COST_LA, None, bm, am, distinct=distinct,
                                        subarrays=T, sub_mult=sm)
                b = brute.BruteFilter(M, c, k, "la", 3.5, bm, am, distinct=distinct, subarrays=T, sub_mult=sm)
                keys = workload.positive_keys(rnd.getrandbits(32), 40)
                assert [int(v) for v in o.envelope(keys)] == b.envelope_words(keys)


def test_envelope_is_tight_at_low_load():
    """Not vacuous: at a light load, where few keys share a block, the
    envelope of c = 2 holds close to twice the sequential filter's bits, and
    it never is all ones."""
    M, k = 1 << 14, 11
    keys = workload.positive_keys(41, 2000)
    f = oracle.OracleFilter(M, 2, k, oracle.COST_LA, None, seed=41)
    f.insert(keys)
    env = f.envelope(keys)
    assert not np.any(f.words & ~env)
    ratio = _popcount(env) / _popcount(f.words)
    assert 1.95 < ratio <= 2.0, ratio
    assert _popcount(env) < 512 * M // 10


# ------------------------------------------------------- load histogram
# App. C, load histogram figure: the number of blocks per count of set bits.

def test_block_loads_of_empty_and_full_filter():
    f = oracle.OracleFilter(37, 2, 8, oracle.COST_EXP, None, seed=2)
    h = f.block_loads()
    assert h[0] == 37 and h.sum() == 37
    full = np.full(8 * 37, np.uint64((1 << 64) - 1), dtype=np.uint64)
    h = f.block_loads(full)
    assert h[512] == 37 and h.sum() == 37


@pytest.mark.parametrize("M,c,kind", [(1, 2, "exp"), (5, 1, "none"), (12, 3, "mix"), (64, 2, "la")])
def test_block_loads_match_set_counts(M, c, kind):
    """Equal to counting |F'| over the set-based blocks after the same inserts;
    the counts sum to M and the loads to the filter's popcount."""
    rnd = random.Random(M * 10 + c)
    k = 9
    kid = oracle.COST_NAMES[kind]
    par = oracle.default_param(kid, k)
    bm = workload.draw_multipliers(rnd.getrandbits(32), c, coprime_to=M)
    am = workload.draw_multipliers(rnd.getrandbits(32), k)
    o = oracle.OracleFilter(M, c, k, kid, par, bm, am)
    b = brute.BruteFilter(M, c, k, kind, par, bm, am)
    for x in workload.positive_keys(rnd.getrandbits(32), 30 * M):
        o.insert_one(int(x))
        b.insert(int(x))
    h = o.block_loads()
    want = np.zeros(513, dtype=np.uint64)
    for P, cnt in b.load_counts().items():
        want[P] = cnt
    assert np.array_equal(h, want)
    assert int(h.sum()) == M
    assert int((np.arange(513, dtype=np.uint64) * h).sum()) == _popcount(o.words)


def test_block_loads_of_random_words():
    rng = np.random.default_rng(5)
    M = 300
    words = _random_words(rng, 8 * M, 0.37)
    f = oracle.OracleFilter(M, 1, 4, oracle.COST_NONE, None, seed=1)
    h = f.block_loads(words)
    per_block = np.bitwise_count(words.reshape(M, 8)).sum(axis=1)
    assert np.array_equal(h, np.bincount(per_block, minlength=513).astype(np.uint64))
    assert int((np.arange(513, dtype=np.uint64) * h).sum()) == _popcount(words)


# ---------------------------------------------------- mixed cost (sigma)
# App. A eq. cost:mix: sigma k (j/512)^k / (1/2)^k + a, the local FPR of the
# block relative to the target FPR at half load, weighted by sigma k.

@pytest.mark.parametrize("sigma", [2.5, 50.0])
@pytest.mark.parametrize("k", [7, 8, 10, 14])
def test_mix_cost_at_half_load_is_sigma_k_plus_a(sigma, k):
    for a in range(k + 1):
        assert oracle.cost(oracle.COST_MIX, sigma, k, 256, a) == sigma * k + a


@pytest.mark.parametrize("sigma", [Fraction(5, 2), Fraction(50), Fraction(3, 4)])
@pytest.mark.parametrize("k", [7, 10, 14])
def test_mix_cost_against_exact_rational_value(sigma, k):
    """The double cost is within a few ulp of sigma k (j/512)^k 2^k + a
    evaluated in exact rational arithmetic."""
    for j in range(1, 513, 11):
        for a in (0, 1, k // 2, k):
            exact = sigma * k * Fraction(j, 512) ** k * 2 ** k + a
            got = oracle.cost(oracle.COST_MIX, float(sigma), k, j, a)
            assert got == pytest.approx(float(exact), rel=1e-14, abs=0)


@pytest.mark.parametrize("k", [7, 14])
def test_mix_fpr_term_scales_with_sigma(k):
    """With a = 0 the cost is the FPR term alone: MIX_sigma = sigma MIX_1."""
    for sigma in (2.5, 50.0):
        for j in range(1, 513, 7):
            one = oracle.cost(oracle.COST_MIX, 1.0, k, j, 0)
            assert oracle.cost(oracle.COST_MIX, sigma, k, j, 0) == pytest.approx(sigma * one, rel=1e-15)


# ------------------------------------ conditional FPR with several choices
# Section 4.1 (the FPR of a filter follows from its block contents): for a
# never-inserted key, the probability that all k addresses fall inside one
# of its candidates, given what those candidates hold.

@pytest.mark.parametrize("c", [2, 3, 4])
@pytest.mark.parametrize("distinct", [False, True])
def test_conditional_fpr_of_single_block(c, distinct):
    """M = 1: every candidate is the same block of P set bits, so the
    estimate is (P/512)^k (random addresses) or C(P,k)/C(512,k) (distinct),
    whatever c is."""
    k = 5
    rng = np.random.default_rng(c)
    for density in (0.1, 0.5, 0.93):
        f = oracle.OracleFilter(1, c, k, oracle.COST_EXP, None, [(1 << 33) | 1] * c,
                                workload.draw_multipliers(7, k), distinct=distinct)
        words = _random_words(rng, 8, density)
        P = _popcount(words)
        want = (P / 512) ** k if not distinct else math.comb(P, k) / math.comb(512, k)
        got = f.conditional_fpr(workload.negative_keys(3, 10, 50), words)
        assert got == pytest.approx(want, rel=1e-13)


def _enumerated_fpr(sets: list[np.ndarray], k: int, distinct: bool) -> float:
    """Probability over all ordered address pairs (k = 2) or single addresses
    (k = 1) that the key's addresses lie inside one of the given blocks."""
    A = np.stack(sets, axis=1).astype(np.int64)  # 512 x c: address in block i
    if k == 1:
        return float(A.any(axis=1).sum()) / 512
    inside = (A @ A.T) > 0  # (f1, f2) both inside some block
    hits = int(inside.sum())
    if not distinct:
        return hits / 512 ** 2
    return (hits - int(np.trace(inside))) / (512 * 511)


def _block_sets(words: np.ndarray, b: int) -> np.ndarray:
    blk = words[8 * b:8 * b + 8]
    return np.array([(int(blk[f // 64]) >> (f % 64)) & 1 for f in range(512)], dtype=bool)


@pytest.mark.parametrize("c", [2, 3, 4])
@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_conditional_fpr_equals_pair_enumeration(c, M):
    """Tiny filters (M <= 4) with random block contents: the inclusion-
    exclusion estimate equals exact enumeration over all 512^2 address pairs
    (k = 2) and all 512 addresses (k = 1), for both bit selections. Keys
    whose candidates coincide and keys whose candidates differ both occur."""
    rng = np.random.default_rng(10 * M + c)
    rnd = random.Random(M + 100 * c)
    for k in (1, 2):
        for distinct in (False, True) if k == 2 else (False,):
            words = np.concatenate([_random_words(rng, 8, d) for d in rng.uniform(0.2, 0.9, size=M)])
            bm = workload.draw_multipliers(rnd.getrandbits(32), c, coprime_to=M)
            f = oracle.OracleFilter(M, c, k, oracle.COST_LA, None, bm, workload.draw_multipliers(9, k),
                                    distinct=distinct)
            keys = workload.positive_keys(rnd.getrandbits(32), 24)
            sets = [_block_sets(words, b) for b in range(M)]
            want = []
            for x in keys:
                cand = [brute.lin_hash(int(a), int(x), M) for a in bm]
                want.append(_enumerated_fpr([sets[b] for b in cand], k, distinct))
            got = f.conditional_fpr(keys, words)
            assert got == pytest.approx(float(np.mean(want)), rel=1e-12)
            for x, w in zip(keys[:6], want):
                assert f.conditional_fpr([x], words) == pytest.approx(w, rel=1e-12)


# ------------------------------------------------------------ placement
# Sections 3.1 and 3.2: each insert either finds F(x) in a candidate and
# writes nothing, or sets F(x) in exactly one candidate. A build is then fixed
# by its per-key decisions; the placement comparator rebuilds it from them.

@pytest.mark.parametrize("M,c,k,kind,distinct", [(97, 2, 11, oracle.COST_LA, False),
                                                  (1 << 10, 3, 8, oracle.COST_MIX, False),
                                                  (6, 2, 14, oracle.COST_EXP, True),
                                                  (1, 4, 5, oracle.COST_EXP, False),
                                                  (3000, 1, 9, oracle.COST_NONE, False)])
def test_placement_of_the_sequential_decisions_is_the_sequential_filter(M, c, k, kind, distinct):
    """The sequential oracle's own decisions, placed, give its filter word
    for word, also when the keys are placed in another order (the OR does not
    depend on it)."""
    keys = workload.positive_keys(M + c, 4000)
    f = oracle.OracleFilter(M, c, k, kind, None, seed=7, distinct=distinct)
    dec = f.insert_recording(keys)
    assert set(np.unique(dec)) <= set(range(c)) | {0xFF}
    assert np.array_equal(f.place(keys, dec), f.words)
    perm = np.random.default_rng(M).permutation(len(keys))
    assert np.array_equal(f.place(keys[perm], dec[perm]), f.words)


@pytest.mark.parametrize("M,c", [(5, 2), (8, 3), (12, 4), (64, 2)])
def test_placement_equals_set_restatement(M, c):
    """Arbitrary decisions (every candidate index, and 'present'), placed by
    the oracle and by the set-based restatement, word for word."""
    k = 6
    bm = workload.draw_multipliers(40 + M, c, coprime_to=M)
    am = workload.draw_multipliers(41 + M, k)
    keys = workload.positive_keys(M, 300)
    rng = np.random.default_rng(M * c)
    dec = rng.integers(0, c + 1, size=len(keys)).astype(np.uint8)
    dec[dec == c] = 0xFF
    f = oracle.OracleFilter(M, c, k, oracle.COST_MIX, None, bm, am)
    b = brute.BruteFilter(M, c, k, "mix", 2.5, bm, am)
    assert [int(v) for v in f.place(keys, dec)] == b.placed_words(keys, dec)


def test_placement_by_residue_classes_partitions_the_filter():
    """Placing one residue class of blocks at a time writes only that class,
    and the classes together give the whole placement."""
    M, c, k, mod = 1 << 12, 2, 11, 7
    keys = workload.positive_keys(9, 20000)
    f = oracle.OracleFilter(M, c, k, oracle.COST_LA, None, seed=9)
    dec = f.insert_recording(keys)
    whole = f.place(keys, dec)
    acc = np.zeros_like(whole)
    blk = np.arange(M)
    for rem in range(mod):
        part = f.place(keys, dec, part_mod=mod, part_rem=rem).reshape(M, 8)
        assert not part[blk % mod != rem].any()
        assert np.array_equal(part[blk % mod == rem], whole.reshape(M, 8)[blk % mod == rem])
        acc |= part.reshape(-1)
    assert np.array_equal(acc, whole)


def test_placement_detects_a_wrong_or_doubled_candidate():
    """A decision naming the other candidate, or a key whose bits also appear
    in its second candidate, changes the placement: the comparator sees the
    faults a racing insert must not make."""
    M, c, k = 1 << 10, 2, 11
    keys = workload.positive_keys(11, 3000)
    f = oracle.OracleFilter(M, c, k, oracle.COST_LA, None, seed=11)
    dec = f.insert_recording(keys)
    t = int(np.flatnonzero(dec == 0)[0])
    wrong = dec.copy()
    wrong[t] = 1
    assert not np.array_equal(f.place(keys, wrong), f.words)
    doubled = f.words.copy()
    b2 = oracle.block_index(M, 1, 0, int(f.block_mult[1]), int(keys[t]))
    doubled[8 * b2:8 * b2 + 8] |= oracle.mask(f.bit_mult, int(keys[t]))
    assert not np.array_equal(f.place(keys, dec), doubled)
