"""Parity of the HIP path with the sequential oracle (GPU only).

Every check runs the kernels through the C ABI and compares with the oracle
on the same seeded inputs:

* query: bit-exact on filters the oracle built (uploaded to the device);
* deterministic insert: filter words bit-exact with the oracle's;
* racing insert with one choice: bit-exact (the result is order-free);
* racing insert with choices: every key's recorded decision names one of
  its candidates (or "present"), and the filter equals, word for word, the
  oracle's placement of each key's mask into the candidate it names; every
  "present" key is held by a candidate; zero false negatives; every set bit
  lies in the oracle's envelope (each key's mask in all of its candidates);
  and the false-positive rate is within 2% relative of the oracle's
  sequential build.
"""

import math

import numpy as np
import pytest

import oracle
import paper_2501_18977_amd as bbfc
import workload

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

COSTS = {"none": oracle.COST_NONE, "mix": oracle.COST_MIX, "la": oracle.COST_LA, "exp": oracle.COST_EXP}


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def to_dev(a: np.ndarray, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(dev)


def from_dev(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def make_pair(M, c, k, cost, seed):
    bm = workload.draw_multipliers(seed, c, coprime_to=M)
    am = workload.draw_multipliers(seed + 7919, k)
    ref = oracle.OracleFilter(M, c, k, COSTS[cost], None, bm, am)
    gpu = bbfc.Filter(M, c, k, cost, block_mult=bm, bit_mult=am)
    return ref, gpu


# (M, c, k, cost, keys): every hash mode (M = 1, 2^s, even, odd), c = 1..4,
# all costs, k from 1 to 32, loads from light to overloaded.
SMALL_CONFIGS = [
    (1, 2, 5, "exp", 40),
    (8, 3, 6, "mix", 300),
    (1 << 10, 2, 14, "la", 16 * 1024 // 16 * 32),
    (3000, 3, 8, "mix", 3000 * 512 // 12),
    (1001, 2, 11, "exp", 1001 * 512 // 16),
    (1 << 15, 1, 10, "none", (1 << 15) * 512 // 16),
    (777, 4, 20, "la", 777 * 512 // 24),
    (1 << 12, 2, 32, "exp", (1 << 12) * 512 // 48),
    (1 << 12, 2, 1, "exp", 20000),
    (6, 2, 7, "la", 500),
]


def test_device_keys_match_numpy_generator(dev):
    got = from_dev(workload.device_keys(99, 12345, 100003, device=dev))
    want = workload.splitmix64_keys(99, 12345, 100003)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("early", [1, 0])
@pytest.mark.parametrize("M,c,k,cost,n", SMALL_CONFIGS)
def test_query_bits_match_oracle_on_oracle_built_filter(dev, M, c, k, cost, n, early):
    ref, gpu = make_pair(M, c, k, cost, seed=M + 31 * c + k)
    try:
        gpu.set_option(bbfc.OPT_QUERY_EARLY_EXIT, early)
        assert gpu.get_option(bbfc.OPT_QUERY_EARLY_EXIT) == early
        keys = workload.positive_keys(M + k, n)
        ref.insert(keys)
        gpu.upload(ref.words)
        probe = np.concatenate([keys, workload.negative_keys(M + k, n, n + 4321)])
        got = from_dev(gpu.query(to_dev(probe, dev)))
        want = ref.query_bits(probe)
        assert np.array_equal(got, want)
        assert bbfc.unpack_bits(got, len(probe))[:n].all()
    finally:
        gpu.close()


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 4097])
def test_query_ragged_sizes(dev, n):
    ref, gpu = make_pair(257, 2, 9, "exp", seed=n)
    try:
        ref.insert(workload.positive_keys(5, 3000))
        gpu.upload(ref.words)
        probe = np.concatenate([workload.positive_keys(5, n // 2), workload.negative_keys(5, 3000, n - n // 2)])
        out = torch.full((n // 64 + 3,), -1, dtype=torch.int64, device=dev)
        gpu.query(to_dev(probe, dev), out=out)
        got = from_dev(out)
        want = ref.query_bits(probe)
        nw = (n + 63) // 64
        assert np.array_equal(got[:nw], want)
        assert np.all(got[nw:] == np.uint64(2**64 - 1)), "wrote past ceil(n/64) words"
    finally:
        gpu.close()


def test_empty_calls_are_noops(dev):
    gpu = bbfc.Filter(64, 2, 8, "la", seed=1)
    try:
        empty = torch.empty(0, dtype=torch.int64, device=dev)
        out = torch.full((2,), 7, dtype=torch.int64, device=dev)
        gpu.insert(empty)
        gpu.insert_deterministic(empty)
        gpu.query(empty, out=out)
        assert from_dev(out).tolist() == [7, 7]
        assert not gpu.download().any()
    finally:
        gpu.close()


@pytest.mark.parametrize("M,c,k,cost,n", SMALL_CONFIGS)
def test_deterministic_insert_is_bit_exact(dev, M, c, k, cost, n):
    ref, gpu = make_pair(M, c, k, cost, seed=3 * M + c + k)
    try:
        keys = workload.positive_keys(2 * M + k, n)
        keys = np.concatenate([keys, keys[: n // 10]])  # repeats take the already-present rule
        ref.insert(keys)
        split = len(keys) // 3
        gpu.insert_deterministic(to_dev(keys[:split], dev))
        gpu.insert_deterministic(to_dev(keys[split:], dev))
        got = gpu.download()
        assert np.array_equal(got, ref.words)
    finally:
        gpu.close()


# The sequential insert holds 1024 keys at a time and refills as keys are
# decided: here with every key in conflict (8 blocks), with blocks that share a
# claim-table entry (block indices 8192 apart), and over many refills.
@pytest.mark.parametrize(
    "M,c,k,cost,n",
    [
        (8, 2, 6, "la", 50_000),
        (3 * 8192, 2, 11, "exp", 200_000),
        (1 << 16, 3, 9, "mix", 1 << 20),
        (501, 4, 32, "mix", 20_000),  # the largest LDS: c = 4, k = 32
        (8, 2, 6, "la", 150_000),  # windows of 2^16 keys whose steps leave most keys to the tail
        (1 << 16, 2, 11, "la", 3 * (1 << 16) + 4321),  # several windows and a ragged one
        (1 << 24, 2, 11, "la", 2 * (1 << 18) + 777),  # a large filter's plan: windows of 2^18 keys
        (1 << 14, 4, 20, "la", (1 << 17) + 777),  # four choices through the device-wide steps
        (777, 3, 8, "mix", (1 << 16) + 1),  # odd M, c = 3, one key past a whole window
    ],
)
def test_deterministic_insert_over_many_steps(dev, M, c, k, cost, n):
    ref, gpu = make_pair(M, c, k, cost, seed=5 * M + c + k)
    try:
        keys = workload.positive_keys(M + 3 * k, n)
        print(f"sequential insert M={M} c={c} k={k} n={n}", flush=True)
        ref.insert(keys)
        gpu.insert_deterministic(to_dev(keys, dev))
        assert np.array_equal(gpu.download(), ref.words)
    finally:
        gpu.close()


def test_deterministic_insert_default_parameters_match_oracle_derivation(dev):
    """bbfc_create draws multipliers from SplitMix64 seed 0; the oracle
    derives its own from the same published generator."""
    M, c, k = 3000, 3, 8
    gpu = bbfc.Filter(M, c, k, "mix")
    try:
        bm, am = oracle.derive_multipliers(0, M, c, k)
        assert list(gpu.params.block_mult) == bm and list(gpu.params.bit_mult) == am
        assert gpu.params.cost_param == oracle.default_param(oracle.COST_MIX, k)
        ref = oracle.OracleFilter(M, c, k, oracle.COST_MIX, None, seed=0)
        keys = workload.positive_keys(77, 50000)
        ref.insert(keys)
        gpu.insert_deterministic(to_dev(keys, dev))
        assert np.array_equal(gpu.download(), ref.words)
    finally:
        gpu.close()


@pytest.mark.parametrize("tile", [0, 2])
@pytest.mark.parametrize("M", [1, 64, 1 << 16, 3000, 1001])
def test_one_choice_racing_insert_is_bit_exact(dev, M, tile):
    """With one choice the racing insert is the OR of all masks whatever the
    schedule: bit-exact with the oracle, in tiles of 64 keys (the default,
    every resident wavefront working) and of 8 keys."""
    ref, gpu = make_pair(M, 1, 10, "none", seed=M)
    try:
        gpu.set_option(bbfc.OPT_INSERT_TILE, tile)
        keys = workload.positive_keys(M, 200_000)
        ref.insert(keys)
        gpu.insert(to_dev(keys, dev))
        assert np.array_equal(gpu.download(), ref.words)
    finally:
        gpu.close()


def _fpr_gate(ref, gpu_words, n_keys, seed, dev, gpu):
    """Conditional FPR (low variance) within 2% and raw FP counts within 4
    binomial sigma, over 2^24 disjoint negatives."""
    n_neg = 1 << 24
    neg_d = workload.device_keys(seed, n_keys, n_neg, device=dev)
    neg = from_dev(neg_d)
    est_gpu = ref.conditional_fpr(neg, words=gpu_words)
    est_ref = ref.conditional_fpr(neg)
    rel = abs(est_gpu - est_ref) / est_ref
    hits_gpu = int(bbfc.unpack_bits(from_dev(gpu.query(neg_d)), n_neg).sum())
    hits_ref = ref.count_hits(neg)
    sd = math.sqrt(hits_gpu + hits_ref)
    print(f"conditional FPR gpu={est_gpu:.4e} oracle={est_ref:.4e} rel={rel:.4%}; "
          f"raw FP gpu={hits_gpu} oracle={hits_ref} ({(hits_gpu - hits_ref) / max(sd, 1):+.2f} sigma)", flush=True)
    assert rel < 0.02
    assert abs(hits_gpu - hits_ref) < 4 * sd
    return est_gpu, est_ref


def check_decisions(ref, keys: np.ndarray, dec: np.ndarray, words: np.ndarray) -> None:
    """Validity of a racing build (Sections 3.1, 3.2): each key either found
    F(x) in a candidate (0xFF) or set it in exactly one candidate, the one
    its decision names. So every decision is a candidate index or 0xFF, the
    filter is exactly the oracle's placement of the decided keys' masks, and
    every "present" key is held by some candidate of the final filter."""
    assert len(dec) == len(keys)
    bad = (dec >= ref.c) & (dec != 0xFF)
    assert not bad.any(), f"{int(bad.sum())} decisions name no candidate"
    placed = ref.place(keys, dec)
    diff = np.flatnonzero(placed != words)
    assert len(diff) == 0, f"{len(diff)} words differ from the placement, first at block {diff[0] // 8}"
    chk = oracle.OracleFilter(ref.M, ref.c, ref.k, ref.kind, ref.param, ref.block_mult, ref.bit_mult,
                              distinct=bool(ref.distinct))
    chk.words[:] = words
    present = keys[dec == 0xFF]
    assert chk.query(present).all(), "a key decided 'present' is not held"


RACING_CONFIGS = [
    (1 << 15, 2, 14, "la", 1 << 20),     # 2^20 keys, 16 bits/key, LA
    (1 << 14, 3, 8, "mix", 3 << 18),    # three choices, MIX, ~10.7 bits/key
    (3000, 2, 11, "exp", 3000 * 32),    # even non-power-of-two M, EXP
    (1 << 18, 2, 11, "la", 1 << 23),    # 32768 keys in flight: the tiles of 8 keys on 1024 workgroups
]


@pytest.mark.parametrize("M,c,k,cost,n", RACING_CONFIGS + [
    (777, 4, 20, "la", 777 * 512 // 24),  # four choices, odd M
    (1, 2, 5, "exp", 40),                 # one block: all candidates coincide
    (6, 2, 7, "la", 500),                 # overloaded: many keys find themselves present
    (1 << 12, 2, 32, "exp", 1 << 12 + 7), # k = 32
])
@pytest.mark.parametrize("tile,lpk,tpw", [(1, 8, 1), (1, 8, 2), (1, 4, 1), (1, 4, 2), (2, 8, 1)])
def test_racing_insert_decisions_rebuild_the_filter(dev, M, c, k, cost, n, tile, lpk, tpw):
    """Both racing kernels (tiles of 64 keys in every launch shape, tiles of
    8 keys): the recorded decisions rebuild the filter exactly."""
    ref, gpu = make_pair(M, c, k, cost, seed=c * k + M + lpk + tpw + tile)
    try:
        gpu.set_option(bbfc.OPT_INSERT_TILE, tile)
        gpu.set_shape(bbfc.OP_INSERT, lpk, tpw)
        assert gpu.insert_launch_info(n)["tile_keys"] == (64 if tile == 1 else 8)
        keys_d = workload.device_keys(M + 2, 0, n, device=dev)
        keys = from_dev(keys_d)
        keys = np.concatenate([keys, keys[: n // 8]])  # repeats: decided present or placed again
        dec = gpu.insert_recorded(to_dev(keys, dev)).cpu().numpy()
        check_decisions(ref, keys, dec, gpu.download())
        assert (dec[n:] == 0xFF).mean() > 0.5 or M < 8, "repeated keys should mostly find themselves present"
    finally:
        gpu.close()


def test_racing_insert_decisions_on_top_of_a_filter(dev):
    """A second racing call decides on the first call's blocks: the filter is
    the first build plus the second call's placement."""
    M, c, k = 1 << 12, 3, 9
    ref, gpu = make_pair(M, c, k, "mix", seed=41)
    try:
        a = workload.positive_keys(41, 30000)
        b = workload.negative_keys(41, 30000, 30000)
        gpu.insert(to_dev(a, dev))
        first = gpu.download()
        dec = gpu.insert_recorded(to_dev(b, dev)).cpu().numpy()
        assert np.array_equal(gpu.download(), ref.place(b, dec, words=first))
    finally:
        gpu.close()


@pytest.mark.parametrize("tile", [0, 1])
@pytest.mark.parametrize("M,c,k,cost,n", RACING_CONFIGS)
def test_racing_insert_invariants_and_fpr(dev, M, c, k, cost, n, tile):
    """The default racing insert (tiles of 8 keys at these bounds) and the
    one with tiles of 64 keys: exact validity, zero false negatives, the
    envelope, and the FPR gate against the oracle's sequential build."""
    ref, gpu = make_pair(M, c, k, cost, seed=c * k + M)
    try:
        gpu.set_option(bbfc.OPT_INSERT_TILE, tile)
        assert gpu.insert_launch_info(n)["tile_keys"] == (8 if tile == 0 else 64)
        keys_d = workload.device_keys(M, 0, n, device=dev)
        keys = from_dev(keys_d)
        ref.insert(keys)
        # the recorded kernel has the timed kernel's schedule: its build is
        # checked exactly, then the timed kernel's own build as below
        check_decisions(ref, keys, gpu.insert_recorded(keys_d).cpu().numpy(), gpu.download())
        gpu.clear()
        gpu.insert(keys_d)
        hits = bbfc.unpack_bits(from_dev(gpu.query(keys_d)), n)
        assert hits.all(), f"{(~hits).sum()} false negatives"
        words = gpu.download()
        env = ref.envelope(keys)
        assert not np.any(words & ~env), "a set bit no key could have set"
        # the oracle's own query on the downloaded filter agrees (sampled)
        sample = keys[:: max(1, n // 4096)]
        chk = oracle.OracleFilter(M, c, k, COSTS[cost], None, ref.block_mult, ref.bit_mult)
        chk.words[:] = words
        assert chk.query(sample).all()
        _fpr_gate(ref, words, n, M + 1, dev, gpu)
    finally:
        gpu.close()


def test_upload_download_clear_roundtrip(dev):
    gpu = bbfc.Filter(513, 2, 9, "exp", seed=3)
    try:
        w = workload.splitmix64_keys(1, 0, 8 * 513)
        gpu.upload(w)
        assert np.array_equal(gpu.download(), w)
        gpu.clear()
        assert not gpu.download().any()
    finally:
        gpu.close()


def test_stream_ordering_on_side_stream(dev):
    ref, gpu = make_pair(1 << 12, 2, 12, "la", seed=5)
    try:
        keys = workload.positive_keys(5, 40000)
        ref.insert(keys)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            kd = to_dev(keys, dev)
            gpu.insert_deterministic(kd)
            out = gpu.query(kd)
        s.synchronize()
        assert bbfc.unpack_bits(out.cpu().numpy(), len(keys)).all()
        assert np.array_equal(gpu.download(), ref.words)
    finally:
        gpu.close()


@pytest.mark.parametrize("op", [bbfc.OP_QUERY, bbfc.OP_INSERT])
def test_single_filter_tuner(dev, op):
    ref, gpu = make_pair(1 << 14, 2, 11, "la", seed=9)
    try:
        keys = workload.positive_keys(9, 1 << 18)
        ref.insert(keys)
        gpu.upload(ref.words)
        probe = np.concatenate([keys, workload.negative_keys(9, 1 << 18, 1 << 18)])
        pd = to_dev(probe, dev)
        out = torch.empty((len(probe) + 63) // 64, dtype=torch.int64, device=dev)
        best = gpu.tune(op, pd if op == bbfc.OP_QUERY else to_dev(keys, dev), out=out, reps=1)
        assert best["lanes_per_key"] in (4, 8) and best["tiles_per_wave"] in (1, 2) and best["ms"] > 0
        assert gpu.get_shape(op)["lanes_per_key"] == best["lanes_per_key"]
        assert gpu.get_shape(op)["tiles_per_wave"] == best["tiles_per_wave"]
        other = bbfc.OP_INSERT if op == bbfc.OP_QUERY else bbfc.OP_QUERY
        assert gpu.get_shape(other)["lanes_per_key"] == 8 and gpu.get_shape(other)["tiles_per_wave"] == 1
        assert np.array_equal(gpu.download(), ref.words), "tuning changed the filter"
        assert np.array_equal(from_dev(gpu.query(pd)), ref.query_bits(probe))
        if op == bbfc.OP_INSERT:
            # 2048 keys in flight on this filter: tiles of 8 keys (the
            # default here) are about 3x faster than any shape of 64 keys
            assert gpu.get_option(bbfc.OPT_INSERT_TILE) in (0, 2)
            assert gpu.insert_launch_info(1 << 18)["tile_keys"] == 8
            gpu.set_option(bbfc.OPT_INSERT_TILE, 1)
            gpu.tune(op, to_dev(keys, dev), reps=2)
            assert gpu.get_option(bbfc.OPT_INSERT_TILE) == 2
            assert np.array_equal(gpu.download(), ref.words), "tuning changed the filter"
    finally:
        gpu.close()


@pytest.mark.parametrize("lpk,tpw", [(8, 1), (8, 2), (4, 1), (4, 2)])
def test_query_and_deterministic_parity_in_every_shape(dev, lpk, tpw):
    for M, c, k, cost, n in SMALL_CONFIGS[:6]:
        ref, gpu = make_pair(M, c, k, cost, seed=M + lpk + tpw)
        try:
            gpu.set_shape(bbfc.OP_QUERY, lpk, tpw)
            gpu.set_shape(bbfc.OP_INSERT, lpk, tpw)
            keys = workload.positive_keys(M + 3, n)
            ref.insert(keys)
            gpu.upload(ref.words)
            probe = np.concatenate([keys, workload.negative_keys(M + 3, n, n + 77)])
            assert np.array_equal(from_dev(gpu.query(to_dev(probe, dev))), ref.query_bits(probe))
            if c == 1:
                gpu.clear()
                gpu.insert(to_dev(keys, dev))
                assert np.array_equal(gpu.download(), ref.words)
        finally:
            gpu.close()


def test_option_validation(dev):
    gpu = bbfc.Filter(64, 2, 8, "la", seed=1)
    try:
        assert gpu.get_option(bbfc.OPT_INSERT_INFLIGHT) == 0
        gpu.set_option(bbfc.OPT_INSERT_INFLIGHT, 4096)
        assert gpu.get_option(bbfc.OPT_INSERT_INFLIGHT) == 4096
        assert gpu.get_option(bbfc.OPT_INSERT_TILE) == 0
        gpu.set_option(bbfc.OPT_INSERT_TILE, 2)
        assert gpu.get_option(bbfc.OPT_INSERT_TILE) == 2
        for opt, val in ((bbfc.OPT_QUERY_EARLY_EXIT, 2), (bbfc.OPT_INSERT_INFLIGHT, -1), (bbfc.OPT_INSERT_TILE, 3),
                         (99, 0)):
            with pytest.raises(bbfc.BBFCError):
                gpu.set_option(opt, val)
    finally:
        gpu.close()


def test_key_count_bound(dev):
    """More than 2^56 keys in one call is an argument error, caught before
    anything is launched (the library never reads the buffers here)."""
    lib = bbfc.lib()
    gpu = bbfc.Filter(64, 2, 8, "la", seed=1, subarrays=2)
    try:
        buf = torch.zeros(64, dtype=torch.int64, device=dev)
        big = (1 << 56) + 1
        assert lib.bbfc_insert(gpu.handle, buf.data_ptr(), big, None) == -1
        assert lib.bbfc_insert_deterministic(gpu.handle, buf.data_ptr(), big, None) == -1
        assert lib.bbfc_query(gpu.handle, buf.data_ptr(), big, buf[32:].data_ptr(), None) == -1
        assert lib.bbfc_bulk_insert(gpu.handle, buf.data_ptr(), big, buf.data_ptr(), 8, None) == -1
        assert b"2^56" in lib.bbfc_last_error()
        torch.cuda.synchronize()
    finally:
        gpu.close()


def test_overlapping_output_rejected(dev):
    gpu = bbfc.Filter(64, 2, 8, "la", seed=1)
    try:
        buf = torch.zeros(1024, dtype=torch.int64, device=dev)
        with pytest.raises(bbfc.BBFCError, match="overlaps"):
            gpu.query(buf[:512], out=buf[500:])
    finally:
        gpu.close()


def test_latency_probe(dev):
    """The latency probe: every kind gives a plausible time per step for
    each wavefront, the atomic kinds set bits, and bad arguments are
    rejected before anything runs."""
    buf = torch.zeros(8 * (1 << 15), dtype=torch.int64, device=dev)
    out = torch.zeros(4, dtype=torch.float64, device=dev)
    got = {}
    for kind in (0, 1, 2, 3):
        out.zero_()
        bbfc.probe_latency(buf, kind, out, iters=500)
        torch.cuda.synchronize()
        got[kind] = out.cpu().numpy()
        assert np.all(got[kind] > 20) and np.all(got[kind] < 1e5), (kind, got[kind])
    print("latency ns per step (kind: per wavefront):", {k: np.round(v, 1).tolist() for k, v in got.items()},
          flush=True)
    assert buf.ne(0).any()  # kinds 1 and 2 ORed bits in
    # an atomic with its wait takes longer than no step at all, and a read
    # followed by an atomic longer than the atomic alone
    assert got[2].mean() > got[1].mean() * 0.8
    for kwargs in ({"kind": 4}, {"kind": 0, "iters": 0}):
        with pytest.raises(bbfc.BBFCError):
            bbfc.probe_latency(buf, out=out, **kwargs)
    with pytest.raises(bbfc.BBFCError, match="power-of-two"):
        bbfc.probe_latency(buf[:8 * 7], 0, out)


def test_probes_run(dev):
    buf = torch.zeros(8 * (1 << 16), dtype=torch.int64, device=dev)
    sink = torch.zeros(1 << 16, dtype=torch.int64, device=dev)
    bbfc.probe_gather(buf, 1 << 18, 1, sink)
    bbfc.probe_gather(buf, 1 << 18, 1, sink, access_bytes=128)
    bbfc.probe_insert_pattern(buf, 1 << 18, 0, 3, sink)
    torch.cuda.synchronize()
    assert not buf.any()
    bbfc.probe_insert_pattern(buf, 1 << 18, 11, 4, sink)
    torch.cuda.synchronize()
    ones = int(np.bitwise_count(buf.cpu().numpy().view(np.uint64)).sum())
    assert 0 < ones <= 11 * (1 << 18)
    with pytest.raises(bbfc.BBFCError, match="mask_bits"):
        bbfc.probe_insert_pattern(buf, 1, 33, 4, sink)
    # the same keys and masks under the other schedules set the same number
    # of bits at most, each key's mask in one of its two lines
    for schedule in (0, 1, 2):
        buf.zero_()
        bbfc.probe_insert_schedule(buf, 1 << 18, 11, schedule, 4, sink)
        torch.cuda.synchronize()
        got = int(np.bitwise_count(buf.cpu().numpy().view(np.uint64)).sum())
        assert 0 < got <= 11 * (1 << 18), schedule
    with pytest.raises(bbfc.BBFCError, match="schedule"):
        bbfc.probe_insert_schedule(buf, 1, 11, 3, 4, sink)
    buf.zero_()
    bbfc.probe_atomic64(buf, 1 << 18, 2)
    dst = torch.empty_like(buf)
    bbfc.probe_copy(buf, dst)
    torch.cuda.synchronize()
    assert torch.equal(buf, dst)
    assert int(buf.ne(0).sum()) > 0
    src = torch.arange(1 << 19, dtype=torch.int64, device=dev)
    d64 = torch.zeros_like(src)
    bbfc.probe_copy(src, d64, request_bytes=64)
    torch.cuda.synchronize()
    assert torch.equal(src, d64)
    with pytest.raises(bbfc.BBFCError):
        bbfc.probe_copy(src[:1000], d64[:1000], request_bytes=64)
    with pytest.raises(bbfc.BBFCError):
        bbfc.probe_copy(src, d64, request_bytes=32)


def test_query_concurrent_with_insert_sees_a_subset(dev):
    """An insert and a query of the same filter on two streams at once: bits
    are only ever set, so every answer of the concurrent query is also an
    answer of a query after the insert (the concurrent one sees some subset
    of the in-flight insert), and the later query has no false negatives."""
    M, n = 1 << 16, 1 << 21
    gpu = bbfc.Filter(M, 2, 11, "la", seed=31)
    try:
        keys = workload.device_keys(31, 0, 2 * n, device=dev)  # n inserted, n never inserted
        s_ins, s_q = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(s_ins):
            gpu.insert(keys[:n])
        with torch.cuda.stream(s_q):
            during = gpu.query(keys)
        torch.cuda.synchronize()
        after = gpu.query(keys)
        torch.cuda.synchronize()
        d, a = from_dev(during), from_dev(after)
        assert not np.any(d & ~a), "the concurrent query saw a bit the finished filter does not have"
        assert bbfc.unpack_bits(a, 2 * n)[:n].all()
    finally:
        gpu.close()


@pytest.mark.parametrize("M,c", [(1 << 15, 2), (1 << 15, 3), (3000, 4), (1 << 25, 2), (1 << 15, 1), (1, 2)])
def test_insert_launch_info_realises_the_bound(dev, M, c):
    """The default bound on keys in flight, M/(8(c-1)) (none for one
    choice), is what the launch realises, rounded down to whole wavefronts
    of the tile size the bound selects (8 keys up to 2^16 in flight, else
    64), and never more than the call's keys."""
    gpu = bbfc.Filter(M, c, 11 if c > 1 else 10, "la" if c > 1 else "none", seed=2)
    try:
        n = 1 << 22
        info = gpu.insert_launch_info(n)
        bound = (1 << 62) if c == 1 else max(64, M // (8 * (c - 1)))
        tile = 8 if bound <= 1 << 16 else 64
        assert info["tile_keys"] == tile
        if bound <= info["workgroups"] * 4 * tile:  # the grid holds the bound
            assert info["keys_in_flight"] == max(tile, bound // tile * tile)
        assert info["keys_in_flight"] <= max(bound, tile)
        assert gpu.insert_launch_info(100)["keys_in_flight"] <= 128  # one wide unit holds 64 or 128 keys
        gpu.set_option(bbfc.OPT_INSERT_INFLIGHT, 1000)
        gpu.set_option(bbfc.OPT_INSERT_TILE, 1)
        info = gpu.insert_launch_info(n)
        assert info["tile_keys"] == 64 and info["keys_in_flight"] == 960 and info["workgroups"] == 4
        gpu.set_option(bbfc.OPT_INSERT_TILE, 2)
        info = gpu.insert_launch_info(n)
        assert info["tile_keys"] == 8 and info["keys_in_flight"] == 1000 and info["workgroups"] == 32
    finally:
        gpu.close()
