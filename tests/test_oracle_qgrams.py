"""Pins of the oracle's canonical q-grams (Section 4.3) and of the 2-bit
packing of the input module. CPU only."""

import numpy as np
import pytest

import oracle
import workload

CODE = {"A": 0, "C": 1, "G": 2, "T": 3}
COMP = str.maketrans("ACGT", "TGCA")


def enc(s):
    return np.array([CODE[ch] for ch in s], dtype=np.uint8)


def brute_qgrams(seq: str, seg_len: int, q: int):
    """Restatement with Python strings: int(..., 4) of the window and of its
    reverse complement (reverse the string, swap A<->T, C<->G)."""
    out = []
    for s in range(len(seq) // seg_len):
        seg = seq[s * seg_len:(s + 1) * seg_len]
        for j in range(len(seg) - q + 1):
            w = seg[j:j + q]
            rc = w[::-1].translate(COMP)
            f = int(w.translate(str.maketrans("ACGT", "0123")), 4)
            r = int(rc.translate(str.maketrans("ACGT", "0123")), 4)
            out.append(min(f, r))
    return out


def test_hand_examples():
    # ACG: forward 0*16+1*4+2 = 6; reverse complement CGT = 1*16+2*4+3 = 27
    assert list(oracle.qgrams(enc("ACG"), 1, 3, 3)) == [6]
    # TTT: reverse complement AAA = 0
    assert list(oracle.qgrams(enc("TTT"), 1, 3, 3)) == [0]
    # ACGT is its own reverse complement: 0*64+1*16+2*4+3 = 27
    assert list(oracle.qgrams(enc("ACGT"), 1, 4, 4)) == [27]
    # windows of GATTACA with q = 2: GA(8)/TC(13)->8, AT(3)/AT->3, TT(15)/AA(0)->0,
    # TA(12)/TA->12, AC(1)/GT(11)->1, CA(4)/TG(14)->4
    assert list(oracle.qgrams(enc("GATTACA"), 1, 7, 2)) == [8, 3, 0, 12, 1, 4]


@pytest.mark.parametrize("q", [1, 2, 5, 15, 16, 17, 21, 31, 32])
def test_matches_string_restatement(q):
    rng = np.random.default_rng(q)
    seq = "".join(rng.choice(list("ACGT"), size=600))
    for seg_len in (600, 150, 37, q, q + 1):
        nseg = 600 // seg_len
        got = oracle.qgrams(enc(seq), nseg, seg_len, q)
        assert list(got) == brute_qgrams(seq[:nseg * seg_len], seg_len, q)


def test_segment_shorter_than_q_has_no_windows():
    assert len(oracle.qgrams(enc("ACGTACGT"), 2, 4, 5)) == 0


@pytest.mark.parametrize("q", [3, 20, 31])
def test_reverse_complement_sequence_has_same_qgrams(q):
    """A sequence and its reverse complement contain the same canonical
    q-grams, in reverse order."""
    b = workload.random_bases(q, 1000)
    rc = (3 - b[::-1]).astype(np.uint8)
    a = oracle.qgrams(b, 1, 1000, q)
    r = oracle.qgrams(rc, 1, 1000, q)
    assert np.array_equal(a, r[::-1])
    assert np.all(a < (1 << (2 * q)) if q < 32 else True)


def test_packing_round_trip_and_layout():
    b = workload.random_bases(7, 1000)
    w = workload.pack_2bit(b)
    assert np.array_equal(workload.unpack_2bit(w, 1000), b)
    # first base in the two most significant bits of word 0
    w1 = workload.pack_2bit(enc("TACG"))
    assert int(w1[0]) == (3 << 62) | (0 << 60) | (1 << 58) | (2 << 56)
    # the random genome's packed words are the SplitMix64 stream itself
    assert np.array_equal(workload.genome_packed(3, 640), workload.splitmix64_keys(3, 0, 20))
