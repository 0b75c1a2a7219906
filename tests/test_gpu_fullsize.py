"""The measured workloads at full size, in the launch shapes that are timed
(GPU only).

* Plain filter: 2^30 keys (SplitMix64 counters [0, 2^30) of seed 0) are
  inserted by the racing insert into 2^25 blocks (2 GiB; c = 2, k = 11, LA,
  default multipliers of seed 0). Then the 2^30 keys and 2^30 never-inserted
  keys (counters [2^30, 2^31)) are queried with 8 lanes per key and 2 tiles
  per wavefront, the autotuner's pick on this workload. Checks:
  - every inserted key answers true;
  - 2^20 sampled answers equal the oracle's query of the same keys on the
    downloaded filter;
  - every other query shape, with early exit on and off, writes the same
    answer words;
  - the false-positive rate over the 2^30 negatives equals, within 2%, the
    oracle's conditional estimate for this filter. The estimate is the exact
    hit probability of 2^22 sampled negatives given the blocks' contents.
* DNA q-grams: a 128 Mbp uniform genome, its 127,999,970 canonical 31-mers
  inserted (fused kernel) into 3,000,000 blocks (12 bits per key; c = 3,
  k = 8, MIX). It is then queried with 10^7 reads of 150 bp at 1%
  substitutions and 10^7 random reads. Checks:
  - every genome 31-mer answers true;
  - sampled genome windows, whose 31-mers the oracle extracts itself, are
    all present in the downloaded filter;
  - the answers for 4096 sampled reads of each set equal the oracle's
    (oracle q-grams, oracle query on the downloaded filter).
* Large q-gram build: a 3.1 Gbp genome with 10% planted repeats in a 5.1 GB
  filter (see its test).
* Batch: 256 filters of uneven sizes through a hipGraph of the persistent
  insert and query (see its test).
* Serving: requests of mixed sizes replayed against the 2^30-key filter
  (see its test).
"""

import math

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


def answer_bits(words_host: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Answer bit t of packed words (bit t % 64 of word t // 64) for each t in idx."""
    idx = np.asarray(idx, dtype=np.uint64)
    return ((words_host[idx >> np.uint64(6)] >> (idx & np.uint64(63))) & np.uint64(1)).astype(bool)


def test_plain_filter_2_pow_30_keys(dev):
    N, M, C, K = 1 << 30, 1 << 25, 2, 11
    bm, am = oracle.derive_multipliers(0, M, C, K)
    keys = torch.empty(2 * N, dtype=torch.int64, device=dev)
    workload.device_keys(0, 0, N, out=keys[:N])
    workload.device_keys(0, N, N, out=keys[N:])
    f = bbfc.Filter(M, C, K, "la", seed=0)
    try:
        assert list(f.params.block_mult) == bm and list(f.params.bit_mult) == am
        f.set_shape(bbfc.OP_INSERT, 8, 1)
        f.set_shape(bbfc.OP_QUERY, 8, 2)
        print("plain: 2^30 keys into 2^25 blocks, racing insert 8x1, query 8x2", flush=True)
        f.insert(keys[:N])
        out = f.query(keys)
        torch.cuda.synchronize()
        assert bool(torch.all(out[: N // 64] == -1)), "an inserted key answered false"

        # other shapes and early exit on/off: the same answer words
        out2 = torch.empty_like(out)
        for early in (1, 0):
            f.set_option(bbfc.OPT_QUERY_EARLY_EXIT, early)
            for lpk in (8, 4):
                for tpw in (1, 2):
                    f.set_shape(bbfc.OP_QUERY, lpk, tpw)
                    f.query(keys, out=out2)
                    torch.cuda.synchronize()
                    assert torch.equal(out, out2), (lpk, tpw, early)
        f.set_option(bbfc.OPT_QUERY_EARLY_EXIT, 1)
        del out2

        words = f.download()
        out_h = out.cpu().numpy().view(np.uint64)
        chk = oracle.OracleFilter(M, C, K, oracle.COST_LA, None, bm, am)
        chk.words = words
        # 64 runs of 16384 consecutive counters anywhere in [0, 2^31)
        rng = np.random.default_rng(30)
        for start in rng.integers(0, 2 * N - 16384, size=64):
            idx = np.arange(int(start), int(start) + 16384, dtype=np.uint64)
            sample = workload.splitmix64_keys(0, int(start), 16384)
            assert np.array_equal(answer_bits(out_h, idx), chk.query(sample)), int(start)

        fp = int(np.bitwise_count(out_h[N // 64:]).sum())
        est = chk.conditional_fpr(workload.splitmix64_keys(0, N + 12345, 1 << 22))
        print(f"plain: FPR over 2^30 negatives {fp / N:.4e}, oracle conditional estimate {est:.4e}", flush=True)
        assert fp / N == pytest.approx(est, rel=0.02)
    finally:
        f.close()
        del keys


def test_plain_filter_2_pow_30_racing_against_sequential(dev):
    """The headline filter built three ways from the same 2^30 keys:

    * the racing insert (the timed kernel);
    * the racing insert that records each key's decision: every decision
      names a candidate or 'present', and on the blocks of one residue class
      (block index = 17 mod 64, 2^19 blocks) the filter equals the oracle's
      placement of the decided keys' masks, word for word;
    * the sequential insert (one key at a time in index order).

    The racing filter's false-positive rate must stay within 2% of the
    sequential build's (Section 4.1): the conditional estimate over 2^24
    never-inserted keys within 2% relative, and the raw false-positive counts
    over the 2^30 never-inserted keys within 4 binomial sigma."""
    N, M, C, K = 1 << 30, 1 << 25, 2, 11
    keys = torch.empty(2 * N, dtype=torch.int64, device=dev)
    workload.device_keys(0, 0, N, out=keys[:N])
    workload.device_keys(0, N, N, out=keys[N:])
    f = bbfc.Filter(M, C, K, "la", seed=0)
    try:
        f.set_shape(bbfc.OP_INSERT, 8, 1)
        f.set_shape(bbfc.OP_QUERY, 8, 2)
        ref = oracle.OracleFilter(M, C, K, oracle.COST_LA, None, seed=0)
        assert list(f.params.block_mult) == [int(v) for v in ref.block_mult]

        print("racing vs sequential: racing build", flush=True)
        f.insert(keys[:N])
        fp_race = int(np.bitwise_count(f.query(keys[N:]).cpu().numpy().view(np.uint64)).sum())
        words_race = f.download()

        print("racing vs sequential: recorded racing build", flush=True)
        f.clear()
        dec_d = f.insert_recorded(keys[:N])
        words_rec = f.download()
        dec = dec_d.cpu().numpy()
        del dec_d
        bad = (dec >= C) & (dec != 0xFF)
        assert not bad.any(), f"{int(bad.sum())} decisions name no candidate"
        host_keys = keys[:N].cpu().numpy().view(np.uint64)
        placed = ref.place(host_keys, dec, part_mod=64, part_rem=17).reshape(M, 8)
        sel = np.arange(17, M, 64)
        assert np.array_equal(placed[sel], words_rec.reshape(M, 8)[sel]), "recorded decisions do not rebuild the blocks"
        print(f"racing vs sequential: {int((dec == 0xFF).sum())} keys decided present, "
              f"{len(sel)} blocks rebuilt from the decisions", flush=True)
        del placed, host_keys, dec, words_rec

        print("racing vs sequential: sequential build", flush=True)
        f.clear()
        f.insert_deterministic(keys[:N])
        fp_seq = int(np.bitwise_count(f.query(keys[N:]).cpu().numpy().view(np.uint64)).sum())
        words_seq = f.download()

        neg = workload.splitmix64_keys(0, N + 777, 1 << 24)
        est_race = ref.conditional_fpr(neg, words=words_race)
        est_seq = ref.conditional_fpr(neg, words=words_seq)
        rel = abs(est_race - est_seq) / est_seq
        sd = math.sqrt(fp_race + fp_seq)
        print(f"racing vs sequential: conditional FPR {est_race:.5e} vs {est_seq:.5e} ({rel:.3%}); raw FP over 2^30 "
              f"negatives {fp_race} vs {fp_seq} ({(fp_race - fp_seq) / sd:+.2f} sigma)", flush=True)
        assert rel < 0.02
        assert abs(fp_race - fp_seq) < 4 * sd
    finally:
        f.close()
        del keys


def read_bases(packed: np.ndarray, reads: np.ndarray, length: int) -> np.ndarray:
    """Bases (one per byte) of the given reads of a packed read set."""
    start = reads.astype(np.int64) * length
    word = start // 32
    off = start % 32
    span = (length + 31) // 32 + 1
    padded = np.concatenate([packed, np.zeros(span, dtype=np.uint64)])
    w = padded[word[:, None] + np.arange(span)[None, :]]
    shifts = np.arange(62, -1, -2, dtype=np.uint64)
    b = ((w[:, :, None] >> shifts[None, None, :]) & np.uint64(3)).astype(np.uint8).reshape(len(reads), -1)
    return b[np.arange(len(reads))[:, None], off[:, None] + np.arange(length)[None, :]]


def test_kmer_workload_128_mbp(dev):
    q, L, G, R = 31, 150, 128_000_000, 10_000_000
    n_g = G - q + 1
    M = bbfc.blocks_for(n_g, 12)
    assert M == math.ceil(n_g * 12 / 512) == 3_000_000
    C, K = 3, 8
    genome = workload.device_keys(21, 0, (G + 31) // 32, device=dev)
    reads = workload.device_reads(genome, G, R, L, 0.01, seed=22)
    rnd = workload.device_keys(23, 0, (R * L + 31) // 32, device=dev)
    bm, am = oracle.derive_multipliers(0, M, C, K)
    f = bbfc.Filter(M, C, K, "mix", seed=0)
    try:
        assert list(f.params.block_mult) == bm and list(f.params.bit_mult) == am
        print("kmer: 128 Mbp genome, 3,000,000 blocks, c=3 k=8 MIX, default shapes", flush=True)
        f.insert_kmers(genome, 1, G, q)
        g_out = f.query_kmers(genome, 1, G, q)
        out_p = f.query_kmers(reads, R, L, q)
        out_n = f.query_kmers(rnd, R, L, q)
        torch.cuda.synchronize()
        g_h = g_out.cpu().numpy().view(np.uint64)
        assert np.all(g_h[: n_g // 64] == np.uint64(2**64 - 1))
        assert answer_bits(g_h, np.arange(n_g // 64 * 64, n_g)).all(), "a genome 31-mer answered false"

        chk = oracle.OracleFilter(M, C, K, oracle.COST_MIX, None, bm, am)
        chk.words = f.download()
        g_packed = genome.cpu().numpy().view(np.uint64)
        rng = np.random.default_rng(31)
        for s in rng.integers(0, G - 20_000, size=16):
            bases = workload.unpack_2bit(g_packed[s // 32:(s + 20_000) // 32 + 2], 20_000 + 64)[s % 32:s % 32 + 20_000]
            assert chk.query(oracle.qgrams(bases, 1, len(bases), q)).all(), int(s)

        per = L - q + 1
        for name, packed_d, out in (("reads", reads, out_p), ("random", rnd, out_n)):
            packed = packed_d.cpu().numpy().view(np.uint64)
            sel = np.sort(rng.choice(R, size=4096, replace=False))
            bases = read_bases(packed, sel, L).reshape(-1)
            want = chk.query(oracle.qgrams(bases, len(sel), L, q))
            idx = (sel[:, None].astype(np.uint64) * np.uint64(per) + np.arange(per, dtype=np.uint64)[None, :]).reshape(-1)
            got = answer_bits(out.cpu().numpy().view(np.uint64), idx)
            print(f"kmer: {name}: sampled hit rate {got.mean():.4f}", flush=True)
            assert np.array_equal(got, want), name
    finally:
        f.close()


def test_batch_256_filters(dev):
    """256 filters, key counts log-uniform in [2^10, 2^24] (4.1e8 keys),
    10-16 bits per key, c = 2, EXP; one persistent insert and one persistent
    query replayed from a hipGraph in the shapes the autotuner picks on this
    workload. Every inserted key answers true, every query shape writes the
    same words, and sampled answers of 12 filters equal the oracle's on the
    downloaded filters."""
    specs = workload.batch_specs(3, 256)
    filters, ns, ks, Ms = [], [], [], []
    for f, (n, bits) in enumerate(specs):
        k = int(round(bits * math.log(2)))
        M = max(1, math.ceil(n * bits / 512))
        filters.append(bbfc.Filter(M, 2, k, "exp", seed=f))
        ns.append(n)
        ks.append(k)
        Ms.append(M)
    try:
        total = sum(ns)
        ins = torch.empty(total, dtype=torch.int64, device=dev)
        qry = torch.empty(2 * total, dtype=torch.int64, device=dev)
        ko = 0
        for f, n in enumerate(ns):
            workload.device_keys(1000 + f, 0, n, out=ins[ko:ko + n])
            workload.device_keys(1000 + f, 0, 2 * n, out=qry[2 * ko:2 * ko + 2 * n])
            ko += n
        ins_plan = bbfc.Batch(filters, ns)
        q_plan = bbfc.Batch(filters, [2 * n for n in ns])
        ins_plan.set_shape(bbfc.OP_INSERT, 8, 1, 0, 1)
        q_plan.set_shape(bbfc.OP_QUERY, 8, 1, 0, 16)
        out = torch.empty(q_plan.total_out_words, dtype=torch.int64, device=dev)
        print(f"batch: 256 filters, {total} keys, graph of persistent insert 8x1 and query 8x1 (grabs of 16)", flush=True)
        graph = bbfc.Graph(ins_plan, ins, q_plan, qry, out)
        graph.launch()
        torch.cuda.synchronize()
        out_h = out.cpu().numpy().view(np.uint64)
        for f, n in enumerate(ns):
            w0 = q_plan.out_offsets[f]
            assert answer_bits(out_h, np.arange(w0 * 64, w0 * 64 + n)).all(), f"filter {f}: a false negative"

        out2 = torch.empty_like(out)
        for lpk in (8, 4):
            for tpw in (1, 2):
                for grab in (0, 16):
                    q_plan.set_shape(bbfc.OP_QUERY, lpk, tpw, 0, grab)
                    q_plan.query(qry, out=out2)
                    torch.cuda.synchronize()
                    assert torch.equal(out, out2), (lpk, tpw, grab)

        order = np.argsort(ns)
        pick = list(order[:4]) + list(order[len(order) // 2 - 2:len(order) // 2 + 2]) + list(order[-4:])
        for f in pick:
            f = int(f)
            n, w0 = ns[f], q_plan.out_offsets[f]
            bm, am = oracle.derive_multipliers(f, Ms[f], 2, ks[f])
            chk = oracle.OracleFilter(Ms[f], 2, ks[f], oracle.COST_EXP, None, bm, am)
            chk.words = filters[f].download()
            cnt = min(n, 8192)
            for start in (0, n - cnt, n, 2 * n - cnt):  # first and last positives, first and last negatives
                sample = workload.splitmix64_keys(1000 + f, start, cnt)
                got = answer_bits(out_h, np.arange(w0 * 64 + start, w0 * 64 + start + cnt))
                assert np.array_equal(got, chk.query(sample)), (f, start)
    finally:
        for fl in filters:
            fl.close()


def test_serve_resident_2_pow_30_filter(dev):
    """The serving workload: 3000 requests (sizes log-uniform in [1, 65536],
    half inserted keys) replayed at an offered 4 G keys/s through 4 slots of
    2^20 keys against the 2^30-key filter. Each request's answers equal
    those of one plain query over all the requests' keys, and the oracle's
    on the downloaded filter for 300 sampled requests."""
    n = 1 << 30
    M = n // 32
    f = bbfc.Filter(M, 2, 11, "la", seed=0)
    try:
        keys = workload.device_keys(0, 0, n, device=dev)
        f.insert(keys)
        torch.cuda.synchronize()
        del keys
        sizes, pst, nst = workload.serve_requests(11, 3000, n)
        parts = []
        for s, p, q in zip(sizes, pst, nst):
            npos = (s + 1) // 2
            parts.append(workload.splitmix64_keys(0, p, npos))
            parts.append(workload.splitmix64_keys(0, q, s - npos))
        flat = np.concatenate(parts)
        offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum(sizes)
        arrivals = np.cumsum(np.random.default_rng(5).exponential(len(flat) / len(sizes) / 4e9, size=len(sizes)))
        srv = bbfc.Server(f, n_slots=4, max_batch_keys=1 << 20, max_pending_keys=1 << 27)
        try:
            answers, lat, wall = srv.replay(flat, offs, arrivals)
        finally:
            srv.close()
        print(f"serve: {len(flat)} keys in {wall * 1e3:.1f} ms, p50 {np.percentile(lat, 50):.0f} us, "
              f"p99 {np.percentile(lat, 99):.0f} us", flush=True)
        plain = bbfc.unpack_bits(f.query(torch.from_numpy(flat.view(np.int64)).to(dev)), len(flat))
        words = f.download()
        chk = oracle.OracleFilter(M, 2, 11, oracle.COST_LA, None, *oracle.derive_multipliers(0, M, 2, 11))
        chk.words = words
        sampled = set(np.random.default_rng(6).choice(len(sizes), size=300, replace=False).tolist())
        for i, s in enumerate(sizes):
            a, b = int(offs[i]), int(offs[i + 1])
            got = bbfc.unpack_bits(answers[i], s)
            assert np.array_equal(got, plain[a:b]), i
            assert got[: (s + 1) // 2].all(), i
            if i in sampled:
                assert np.array_equal(got, chk.query(flat[a:b])), i
    finally:
        f.close()


def test_kmer_workload_3100_mbp_with_repeats(dev):
    """The large q-gram build: a 3.1 Gbp uniform genome with 10% planted
    repeats (300-6000 bp copies at 2% divergence), its 3.1e9 canonical
    31-mers inserted into a filter sized for the expected distinct count at
    14 bits per key (80,234,269 blocks, 5.1 GB; c = 3, k = 10, MIX), queried
    with 5e7 reads of 150 bp at 1% substitutions. Sampled genome windows
    (oracle q-grams) are all present in the downloaded filter, and the
    answers of 4096 sampled reads equal the oracle's."""
    q, L, G, R = 31, 150, 3_100_000_000, 50_000_000
    n_g = G - q + 1
    genome = workload.device_keys(21, 0, (G + 31) // 32, device=dev)
    segs = workload.repeat_segments(24, G, 0.1)
    genome = workload.device_plant(genome, G, segs, 0.02, seed=25)
    reads = workload.device_reads(genome, G, R, L, 0.01, seed=22)
    M = bbfc.blocks_for(int(n_g * (1.0 - 0.1 * 0.98 ** q)), 14)
    assert M == 80_234_269
    C, K = 3, 10
    bm, am = oracle.derive_multipliers(0, M, C, K)
    f = bbfc.Filter(M, C, K, "mix", seed=0)
    try:
        print(f"kmer large: {len(segs[0])} planted segments, {M} blocks", flush=True)
        f.insert_kmers(genome, 1, G, q)
        out = f.query_kmers(reads, R, L, q)
        torch.cuda.synchronize()
        chk = oracle.OracleFilter(M, C, K, oracle.COST_MIX, None, bm, am)
        chk.words = f.download()
        g_packed = genome.cpu().numpy().view(np.uint64)
        rng = np.random.default_rng(32)
        for s in rng.integers(0, G - 20_000, size=16):
            bases = workload.unpack_2bit(g_packed[s // 32:(s + 20_000) // 32 + 2], 20_000 + 64)[s % 32:s % 32 + 20_000]
            assert chk.query(oracle.qgrams(bases, 1, len(bases), q)).all(), int(s)
        del g_packed
        per = L - q + 1
        packed = reads.cpu().numpy().view(np.uint64)
        sel = np.sort(rng.choice(R, size=4096, replace=False))
        want = chk.query(oracle.qgrams(read_bases(packed, sel, L).reshape(-1), len(sel), L, q))
        idx = (sel[:, None].astype(np.uint64) * np.uint64(per) + np.arange(per, dtype=np.uint64)[None, :]).reshape(-1)
        got = answer_bits(out.cpu().numpy().view(np.uint64), idx)
        print(f"kmer large: sampled read hit rate {got.mean():.4f}", flush=True)
        assert np.array_equal(got, want)
    finally:
        f.close()
