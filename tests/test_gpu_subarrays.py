"""Sub-array filters (Section 3.4, Parallelization) on the GPU (GPU only).

* every kernel with the sub-array layout: query bit-exact on oracle-built
  filters, deterministic insert bit-exact, racing insert bit-exact with one
  choice and inside the envelope with choices;
* the bulk insert (stable partition by h_0, one wavefront per sub-array in
  LDS) bit-exact with the oracle's sequential build for every hash case of
  T and S, one to three radix passes, ragged sizes, repeated keys, distinct
  bits, c = 1..4, partition counts per tile and per group of tiles, and
  over several calls;
* at 2^26 keys, sampled sub-arrays of the GPU build equal the oracle's
  build of the keys h_0 sends to them, and every key answers true.
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


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(dev)


def from_dev(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def make_pair(M, T, c, k, cost, seed, distinct=False):
    S = M // T
    bm = workload.draw_multipliers(seed, c, coprime_to=S)
    am = workload.draw_multipliers(seed + 7919, k, coprime_to=workload.distinct_moduli(k) if distinct else 512)
    sm = workload.draw_multipliers(seed + 31, 1, coprime_to=T)[0] if T > 1 else 0
    ref = oracle.OracleFilter(M, c, k, oracle.COST_NAMES[cost], None, bm, am, distinct=distinct, subarrays=T,
                              sub_mult=sm if T > 1 else None)
    gpu = bbfc.Filter(M, c, k, cost, block_mult=bm, bit_mult=am, bit_selection="distinct" if distinct else "random",
                      subarrays=T, sub_mult=sm if T > 1 else None)
    assert gpu.params.subarrays == T and gpu.params.sub_mult == (sm if T > 1 else 0)
    return ref, gpu


# (M, T, c, k, cost, n): pow2 / even / odd T and S
CONFIGS = [
    (1 << 14, 1 << 6, 2, 11, "la", (1 << 14) * 32),
    (3000, 12, 3, 8, "mix", 3000 * 40),
    (1001 * 7, 1001, 2, 14, "exp", 1001 * 7 * 24),
    (4096, 4096, 2, 9, "exp", 4096 * 20),
    (6 * 256, 6, 1, 10, "none", 6 * 256 * 30),
    (777 * 4, 4, 4, 20, "la", 777 * 4 * 20),
]


@pytest.mark.parametrize("M,T,c,k,cost,n", CONFIGS)
def test_query_matches_oracle(dev, M, T, c, k, cost, n):
    ref, gpu = make_pair(M, T, c, k, cost, seed=M + T)
    try:
        keys = workload.positive_keys(M + 1, n)
        ref.insert(keys)
        gpu.upload(ref.words)
        probe = np.concatenate([keys, workload.negative_keys(M + 1, n, n + 999)])
        got = from_dev(gpu.query(to_dev(probe, dev)))
        assert np.array_equal(got, ref.query_bits(probe))
    finally:
        gpu.close()


@pytest.mark.parametrize("M,T,c,k,cost,n", CONFIGS)
def test_per_key_inserts(dev, M, T, c, k, cost, n):
    ref, gpu = make_pair(M, T, c, k, cost, seed=2 * M + T)
    try:
        # above 2^16 keys the sequential insert runs its device-wide window steps
        keys = workload.positive_keys(M + 2, min(n, (1 << 16) + 4321))
        gpu.insert_deterministic(to_dev(keys, dev))
        ref.insert(keys)
        assert np.array_equal(gpu.download(), ref.words)
        gpu.clear()
        gpu.insert(to_dev(keys, dev))
        words = gpu.download()
        if c == 1:
            assert np.array_equal(words, ref.words)
        else:
            assert not np.any(words & ~ref.envelope(keys))
        assert bbfc.unpack_bits(from_dev(gpu.query(to_dev(keys, dev))), len(keys)).all()
    finally:
        gpu.close()


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("M,T,c,k,cost,n", [cfg for cfg in CONFIGS if cfg[2] > 1])
def test_racing_insert_decisions_rebuild_the_filter(dev, M, T, c, k, cost, n, tile):
    """The racing insert on sub-array filters, in tiles of 64 and of 8 keys:
    every recorded decision names a candidate inside the key's sub-array or
    "present", and the oracle's placement of the decided keys is the filter
    word for word (Sections 3.1, 3.2, 3.4)."""
    ref, gpu = make_pair(M, T, c, k, cost, seed=4 * M + T + tile)
    try:
        gpu.set_option(bbfc.OPT_INSERT_TILE, tile)
        keys = workload.positive_keys(M + 9, min(n, 1 << 17))
        keys = np.concatenate([keys, keys[: len(keys) // 8]])
        dec = gpu.insert_recorded(to_dev(keys, dev)).cpu().numpy()
        words = gpu.download()
        assert not ((dec >= c) & (dec != 0xFF)).any()
        assert np.array_equal(ref.place(keys, dec), words)
        assert bbfc.unpack_bits(from_dev(gpu.query(to_dev(keys, dev))), len(keys)).all()
    finally:
        gpu.close()


@pytest.mark.parametrize("M,T,c,k,cost,n", [
    (1 << 17, 1 << 9, 2, 11, "la", 3 * (1 << 16) + 4321),  # several windows and a ragged one
    (777 * 4 * 15, 4, 4, 20, "la", (1 << 17) + 777),      # four choices, odd S = 11655
])
def test_sequential_insert_device_wide_windows(dev, M, T, c, k, cost, n):
    """The sequential insert's device-wide steps (inputs of 2^16 keys and
    more) on sub-array filters: bit-exact with the oracle."""
    ref, gpu = make_pair(M, T, c, k, cost, seed=3 * M + T)
    try:
        keys = workload.positive_keys(M + 5, n)
        print(f"sub-array sequential insert M={M} T={T} c={c} k={k} n={n}", flush=True)
        gpu.insert_deterministic(to_dev(keys, dev))
        ref.insert(keys)
        assert np.array_equal(gpu.download(), ref.words)
    finally:
        gpu.close()


# (M, T, c, k, cost, distinct, n): radix passes 0 (T = 1), 1 (T <= 512), 2, 3
BULK = [
    (1 << 14, 1 << 6, 2, 11, "la", False, (1 << 14) * 32 + 777),
    (1 << 16, 1 << 10, 2, 11, "la", False, 3_000_001),
    (3000, 12, 3, 8, "mix", False, 3000 * 40),
    (1001 * 7, 1001, 2, 14, "exp", True, 1001 * 7 * 24),
    (1 << 19, 1 << 19, 2, 9, "exp", False, 1 << 20),           # S = 1: one block per sub-array
    (6 * 1000, 6, 1, 10, "none", False, 6 * 1000 * 30),         # S = 1000 (1024-block staging)
    (777 * 4, 4, 4, 20, "la", False, 777 * 4 * 20),             # S = 777, c = 4
    (1000, 1, 2, 12, "exp", False, 20000),                      # no sub-arrays, M <= 1024
    (1 << 20, 1 << 19, 3, 7, "mix", False, 1 << 21),            # T = 2^19: three radix passes
    (512 * 300, 300, 2, 32, "exp", True, 512 * 300 * 10),       # k = 32, distinct
    (256, 256, 2, 5, "la", False, 1),
    (256, 256, 2, 5, "la", False, 65),
    (1 << 19, 1 << 11, 2, 11, "la", False, 2 * 2048 * 4096 + 12345),  # partition counts groups of 2 tiles
]


@pytest.mark.parametrize("M,T,c,k,cost,distinct,n", BULK)
def test_bulk_insert_is_bit_exact(dev, M, T, c, k, cost, distinct, n):
    ref, gpu = make_pair(M, T, c, k, cost, seed=3 * M + T + k, distinct=distinct)
    try:
        keys = workload.positive_keys(M + k, n)
        if n > 100:
            keys = np.concatenate([keys, keys[: n // 7]])  # repeats take the already-present rule
        print(f"bulk M={M} T={T} c={c} k={k} n={len(keys)}", flush=True)
        ref.insert(keys)
        gpu.bulk_insert(to_dev(keys, dev))
        words = gpu.download()
        assert np.array_equal(words, ref.words)
    finally:
        gpu.close()


def test_bulk_insert_over_several_calls(dev):
    """Sequential semantics carry across calls (and a call of zero keys)."""
    M, T = 1 << 15, 1 << 7
    ref, gpu = make_pair(M, T, 2, 11, "exp", seed=5)
    try:
        keys = workload.positive_keys(5, 1 << 20)
        cuts = [0, 1, 70_000, 70_000, 500_000, 1 << 20]
        ws = torch.empty(gpu.bulk_workspace_bytes(1 << 20), dtype=torch.uint8, device=dev)
        for a, b in zip(cuts, cuts[1:]):
            gpu.bulk_insert(to_dev(keys[a:b], dev), workspace=ws)
        ref.insert(keys)
        assert np.array_equal(gpu.download(), ref.words)
        # bulk on top of per-key inserts
        more = workload.negative_keys(5, 1 << 20, 300_000)
        gpu.insert_deterministic(to_dev(more[:1000], dev))
        gpu.bulk_insert(to_dev(more[1000:], dev), workspace=ws)
        ref.insert(more)
        assert np.array_equal(gpu.download(), ref.words)
    finally:
        gpu.close()


def test_bulk_insert_rejects(dev):
    big = bbfc.Filter(1 << 12, 2, 8, "exp", subarrays=2, seed=1)  # 2048 blocks per sub-array
    plain = bbfc.Filter(1 << 12, 2, 8, "exp", seed=1)
    small = bbfc.Filter(1 << 12, 2, 8, "exp", subarrays=16, seed=1)
    try:
        keys = to_dev(workload.positive_keys(1, 1000), dev)
        for f in (big, plain):
            with pytest.raises(bbfc.BBFCError) as e:
                f.bulk_insert(keys)
            assert e.value.status == -4
        need = small.bulk_workspace_bytes(1000)
        assert need > 0
        with pytest.raises(bbfc.BBFCError, match="workspace"):
            small.bulk_insert(keys, workspace=torch.empty(need - 1, dtype=torch.uint8, device=dev))
        small.bulk_insert(keys[:0])
        assert not small.download().any()
    finally:
        for f in (big, plain, small):
            f.close()


def test_bulk_insert_sampled_at_scale(dev):
    """2^26 keys into 2^21 blocks in sub-arrays of 256 blocks (2^13 of them):
    eight sampled sub-arrays equal the oracle's build of exactly the keys
    h_0 sends there, in order; every key answers true."""
    n, M, S = 1 << 26, 1 << 21, 256
    T = M // S
    f = bbfc.Filter(M, 2, 11, "la", seed=9, subarrays=T)
    try:
        keys = workload.device_keys(9, 0, n, device=dev)
        f.bulk_insert(keys)
        assert bbfc.unpack_bits(from_dev(f.query(keys)), n).all()
        words = f.download()
        host = from_dev(keys)
        sm = f.params.sub_mult
        # route with the paper's h_0 for T = 2^13: the top 13 bits of a*x mod 2^64
        h0 = (host * np.uint64(sm)) >> np.uint64(64 - 13)
        rng = np.random.default_rng(9)
        for v in rng.choice(T, size=8, replace=False):
            mine = host[h0 == v]
            ref = oracle.OracleFilter(S, 2, 11, oracle.COST_LA, None, list(f.params.block_mult),
                                      list(f.params.bit_mult))
            ref.insert(mine)
            assert np.array_equal(words[8 * S * v:8 * S * (v + 1)], ref.words), int(v)
    finally:
        f.close()
