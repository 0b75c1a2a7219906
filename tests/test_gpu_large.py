"""Large sizes (GPU only): 64-bit block and key indexing.

* a filter of 2^30 + 1 blocks (64 GiB, odd M): the deterministic insert's
  touched blocks equal the oracle's word for word (read back block by block),
  and queries match the oracle bit for bit;
* one query call of 2^32 + 2^16 keys: the answers past index 2^32 are right;
* one bulk insert call of more than 2^31 keys (split into pieces): sampled
  sub-arrays equal the oracle's sequential build.
The oracle's filter array is allocated lazily by the OS, so only the touched
blocks take host memory.
"""

import ctypes

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


def read_block(hip, words_ptr: int, b: int) -> np.ndarray:
    out = np.zeros(8, dtype=np.uint64)
    rc = hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(words_ptr + b * 64), ctypes.c_size_t(64),
                       ctypes.c_int(2))  # device to host
    assert rc == 0
    return out


def test_filter_beyond_2_pow_32_words(dev):
    M, c, k = (1 << 30) + 1, 2, 11
    bm = workload.draw_multipliers(71, c, coprime_to=M)
    am = workload.draw_multipliers(72, k)
    ref = oracle.OracleFilter(M, c, k, oracle.COST_LA, None, bm, am)
    f = bbfc.Filter(M, c, k, "la", block_mult=bm, bit_mult=am)
    try:
        keys = np.concatenate([workload.positive_keys(71, 20_000),
                               np.array([0, 1, 2**64 - 1, 2**63], dtype=np.uint64)])
        f.insert_deterministic(to_dev(keys, dev))
        ref.insert(keys)
        torch.cuda.synchronize()
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.restype = ctypes.c_int
        blocks = sorted({oracle.hash_(a, int(x), M) for x in keys for a in bm})
        assert blocks[-1] > (1 << 29), "no key reached the upper half of the filter"
        wp = f.words_ptr
        for b in blocks:
            assert np.array_equal(read_block(hip, wp, b), ref.words[8 * b:8 * b + 8]), b
        probe = np.concatenate([keys, workload.negative_keys(71, len(keys), 1 << 20)])
        assert np.array_equal(from_dev(f.query(to_dev(probe, dev))), ref.query_bits(probe))
    finally:
        f.close()


def test_query_call_beyond_2_pow_32_keys(dev):
    M, n_pos = 1 << 20, 1 << 16
    f = bbfc.Filter(M, 2, 11, "la", seed=3)
    try:
        pos = workload.device_keys(3, 0, n_pos, device=dev)
        f.insert(pos)
        n = (1 << 32) + n_pos
        keys = torch.empty(n, dtype=torch.int64, device=dev)
        workload.device_keys(3, n_pos, 1 << 32, out=keys[: 1 << 32])  # never inserted
        keys[1 << 32:] = pos
        out = f.query(keys)
        torch.cuda.synchronize()
        assert out.numel() == n // 64
        tail = out[(1 << 32) // 64:]
        assert bool(torch.all(tail == -1)), "an inserted key past index 2^32 answered false"
        del keys
        # the negatives' false positives: the popcount of the first 2^26 words
        head = out[: (1 << 32) // 64]
        ones = 0
        for part in torch.split(head, 1 << 22):
            ones += int(np.bitwise_count(part.cpu().numpy().view(np.uint64)).sum())
        fpr = ones / float(1 << 32)
        print(f"FPR of 2^32 negatives on a 2^16-key, 2^20-block filter: {fpr:.3e}", flush=True)
        assert fpr < 1e-6
    finally:
        f.close()


def test_bulk_insert_beyond_2_pow_31_keys(dev):
    """One bulk insert call of 2^31 + 2^20 + 7 keys, which the library splits
    into pieces of at most 2^31 keys (32-bit offsets inside a piece), into
    2^14 sub-arrays of 256 blocks: every key answers true, and four sampled
    sub-arrays equal the oracle's build of exactly the keys h_0 routes there,
    in index order, across the piece boundary."""
    n = (1 << 31) + (1 << 20) + 7
    T, S = 1 << 14, 256
    M = T * S
    f = bbfc.Filter(M, 2, 11, "la", seed=13, subarrays=T)
    try:
        keys = workload.device_keys(13, 0, n, device=dev)
        f.bulk_insert(keys)
        hits = f.query(keys)
        torch.cuda.synchronize()
        full = n // 64
        assert bool(torch.all(hits[:full] == -1)), "an inserted key answered false"
        assert bbfc.unpack_bits(hits[full:].cpu().numpy(), n - full * 64).all()
        del hits
        words = f.download()
        sm = f.params.sub_mult
        # the paper's h_0 for T = 2^14: the top 14 bits of sub_mult * x mod 2^64
        sm_signed = sm - (1 << 64) if sm >= (1 << 63) else sm
        h0 = ((keys * sm_signed) >> 50) & (T - 1)
        rng = np.random.default_rng(13)
        for v in rng.choice(T, size=4, replace=False):
            # masked selection in chunks below 2^31 elements, in index order
            mine = np.concatenate([part[hp == int(v)].cpu().numpy().view(np.uint64)
                                   for part, hp in zip(torch.split(keys, 1 << 30), torch.split(h0, 1 << 30))])
            assert len(mine) > 100_000
            ref = oracle.OracleFilter(S, 2, 11, oracle.COST_LA, None, list(f.params.block_mult),
                                      list(f.params.bit_mult))
            ref.insert(mine)
            assert np.array_equal(words[8 * S * int(v):8 * S * (int(v) + 1)], ref.words), int(v)
        del keys, h0
    finally:
        f.close()
