"""DNA q-gram keys on the GPU against the oracle (GPU only).

* extraction: bbfc_kmer_keys bit-exact with the oracle's q-grams, which the
  oracle computes from one base per byte (no 2-bit arithmetic shared);
* fused query: answers bit-exact with the oracle querying its own q-grams
  on an oracle-built filter;
* fused insert: bit-exact for one choice; zero false negatives and every
  bit inside the envelope with choices;
* end to end: reads sampled without errors from a genome all answer true
  after the genome's q-grams were inserted; with 1% substitutions the hit
  rate is that of error-free q-grams plus false positives.
"""

import numpy as np
import pytest

import oracle
import paper_2501_18977_amd as bbfc
import workload

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(dev)


def from_dev(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("q", [1, 2, 7, 15, 16, 17, 21, 31, 32])
@pytest.mark.parametrize("n_seg,seg_len", [(1, 100_003), (400, 150), (97, 33), (5, 31), (3, 10)])
def test_extraction_matches_oracle(dev, q, n_seg, seg_len):
    bases = workload.random_bases(q * 1000 + seg_len, n_seg * seg_len)
    seq = to_dev(workload.pack_2bit(bases), dev)
    want = oracle.qgrams(bases, n_seg, seg_len, q)
    assert bbfc.kmer_count(n_seg, seg_len, q) == len(want)
    got = from_dev(bbfc.kmer_keys(seq, n_seg, seg_len, q))
    assert np.array_equal(got[:len(want)], want)


@pytest.mark.parametrize("shape", [(8, 1), (8, 2), (4, 1), (4, 2)])
@pytest.mark.parametrize("c,cost", [(3, "mix"), (2, "la"), (1, "none")])
def test_fused_query_matches_oracle(dev, c, cost, shape):
    q = 31
    genome = workload.random_bases(11, 200_000)
    gkeys = oracle.qgrams(genome, 1, len(genome), q)
    M = bbfc.blocks_for(len(gkeys), 12)
    bm = workload.draw_multipliers(12, c, coprime_to=M)
    am = workload.draw_multipliers(13, 8)
    ref = oracle.OracleFilter(M, c, 8, oracle.COST_NAMES[cost], None, bm, am)
    ref.insert(gkeys)
    f = bbfc.Filter(M, c, 8, cost, block_mult=bm, bit_mult=am)
    try:
        f.set_shape(bbfc.OP_QUERY, *shape)
        f.upload(ref.words)
        # reads: copies of genome windows (positives) and random sequence
        starts = np.random.default_rng(1).integers(0, len(genome) - 150, size=300)
        reads = np.concatenate([genome[s:s + 150] for s in starts] + [workload.random_bases(99, 300 * 150)])
        rk = oracle.qgrams(reads, 600, 150, q)
        got = from_dev(f.query_kmers(to_dev(workload.pack_2bit(reads), dev), 600, 150, q))
        assert np.array_equal(got, ref.query_bits(rk))
        assert bbfc.unpack_bits(got, len(rk))[:300 * 120].all()
    finally:
        f.close()


@pytest.mark.parametrize("tile,shape", [(0, (8, 1)), (1, (8, 1)), (1, (4, 2)), (2, (8, 1))])
@pytest.mark.parametrize("c,cost", [(1, "none"), (3, "mix")])
def test_fused_insert(dev, c, cost, tile, shape):
    """The racing insert of fused q-grams in tiles of 64 keys (two launch
    shapes) and of 8 keys (tile 2, and the default for c = 3 at this size):
    bit-exact with one choice, inside the envelope with three, and every
    q-gram answers true."""
    q = 31
    genome = workload.random_bases(21, 300_000)
    gkeys = oracle.qgrams(genome, 1, len(genome), q)
    M = bbfc.blocks_for(len(gkeys), 12)
    bm = workload.draw_multipliers(22, c, coprime_to=M)
    am = workload.draw_multipliers(23, 8)
    ref = oracle.OracleFilter(M, c, 8, oracle.COST_NAMES[cost], None, bm, am)
    f = bbfc.Filter(M, c, 8, cost, block_mult=bm, bit_mult=am)
    try:
        f.set_shape(bbfc.OP_INSERT, *shape)
        f.set_option(bbfc.OPT_INSERT_TILE, tile)
        seq = to_dev(workload.pack_2bit(genome), dev)
        f.insert_kmers(seq, 1, len(genome), q)
        words = f.download()
        ref.insert(gkeys)
        if c == 1:
            assert np.array_equal(words, ref.words)
        else:
            assert not np.any(words & ~ref.envelope(gkeys))
        hits = bbfc.unpack_bits(from_dev(f.query_kmers(seq, 1, len(genome), q)), len(gkeys))
        assert hits.all()
    finally:
        f.close()


def test_end_to_end_reads_from_device_genome(dev):
    """Genome and reads generated on the device: error-free reads all hit;
    with 1% substitutions the q-gram hit rate is 0.99^31 (error-free
    q-grams) plus the false-positive share of the rest."""
    q, n_bases, n_reads, L = 31, 4_000_000, 20_000, 150
    g = workload.device_keys(5, 0, (n_bases + 31) // 32, device=dev)  # packed uniform genome
    n_keys = n_bases - q + 1
    M = bbfc.blocks_for(n_keys, 12)
    f = bbfc.Filter(M, 3, 8, "mix", seed=1)
    try:
        f.insert_kmers(g, 1, n_bases, q)
        clean = workload.device_reads(g, n_bases, n_reads, L, 0.0, seed=7)
        hits = bbfc.unpack_bits(from_dev(f.query_kmers(clean, n_reads, L, q)), n_reads * (L - q + 1))
        assert hits.all(), "an error-free read q-gram was not found"
        noisy = workload.device_reads(g, n_bases, n_reads, L, 0.01, seed=8)
        rate = bbfc.unpack_bits(from_dev(f.query_kmers(noisy, n_reads, L, q)), n_reads * (L - q + 1)).mean()
        rnd = workload.device_keys(77, 0, (n_reads * L + 31) // 32, device=dev)
        fpr = bbfc.unpack_bits(from_dev(f.query_kmers(rnd, n_reads, L, q)), n_reads * (L - q + 1)).mean()
        clean_share = 0.99 ** q
        expect = clean_share + (1 - clean_share) * fpr
        print(f"noisy-read hit rate {rate:.4f}, expected {expect:.4f}; random-read FPR {fpr:.2e}", flush=True)
        assert abs(rate - expect) < 0.01
        assert fpr < 0.02
    finally:
        f.close()


@pytest.mark.parametrize("n,frac", [(200_003, 0.1), (65_536, 0.3), (1_000, 0.0)])
def test_device_planting_matches_numpy(dev, n, frac):
    bases = workload.random_bases(31, n)
    segs = workload.repeat_segments(32, n, frac)
    want = workload.pack_2bit(workload.plant_numpy(bases, segs, 0.02, 33))
    got = from_dev(workload.device_plant(to_dev(workload.pack_2bit(bases), dev), n, segs, 0.02, 33))
    assert np.array_equal(got, want)


def test_kmer_argument_errors(dev):
    seq = torch.zeros(4, dtype=torch.int64, device=dev)
    with pytest.raises(bbfc.BBFCError):
        bbfc.kmer_keys(seq, 1, 100, 33)
    with pytest.raises(bbfc.BBFCError):
        bbfc.kmer_keys(seq, 1, 100, 0)
    assert bbfc.kmer_count(10, 20, 31) == 0
    assert len(bbfc.kmer_keys(seq, 10, 20, 31)) == 0
    f = bbfc.Filter(64, 2, 8, "mix", seed=1)
    try:
        buf = torch.zeros(64, dtype=torch.int64, device=dev)
        with pytest.raises(bbfc.BBFCError, match="overlaps"):
            f.query_kmers(buf[:8], 1, 256, 31, out=buf[7:])  # 226 answers in 4 words, from word 7
        f.query_kmers(buf[:8], 1, 256, 31, out=buf[8:])
    finally:
        f.close()
