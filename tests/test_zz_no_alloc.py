"""The sequential insert without allocation, bbfc_insert_deterministic_noalloc,
against bbfc_insert_deterministic (GPU only).

Both entry points are called through the C ABI on the same keys into two
filters with the same multipliers; the filter words must be identical. Two
calls in a row share the static scratch, the second with fewer keys, so a
window or claim left behind by the first call would show in the second.
Cases: several windows with a ragged one (c = 2), a smaller input with
three choices, a filter of 2^24 blocks (where the allocating insert uses
another window plan), and an input below one window (no scratch).
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


def pair(M, c, k, cost, seed):
    bm = workload.draw_multipliers(seed, c, coprime_to=M)
    am = workload.draw_multipliers(seed + 7919, k)
    return (bbfc.Filter(M, c, k, cost, block_mult=bm, bit_mult=am),
            bbfc.Filter(M, c, k, cost, block_mult=bm, bit_mult=am))


# in order: each call after the first has fewer keys than the one before
CALLS = [
    (1 << 16, 2, 11, "la", 3 * (1 << 16) + 4321),
    (3000, 3, 8, "mix", (1 << 16) + 77),
    (1 << 24, 2, 11, "la", (1 << 16) + 5),
    (777, 4, 20, "la", 20000),
]


def test_two_calls_in_a_row_match_the_allocating_insert(dev):
    for i, (M, c, k, cost, n) in enumerate(CALLS):
        print(f"no-alloc sequential insert: call {i} M={M} c={c} k={k} n={n}", flush=True)
        ref, na = pair(M, c, k, cost, seed=M + c + k)
        try:
            keys = workload.positive_keys(M + k, n)
            kd = torch.from_numpy(keys.view(np.int64)).to(dev)
            ref.insert_deterministic(kd)
            na.insert_deterministic_noalloc(kd)
            torch.cuda.synchronize()
            want = ref.download()
            assert np.array_equal(na.download(), want), f"call {i}: filter words differ"
            if M <= 1 << 16:
                chk = oracle.OracleFilter(M, c, k, oracle.COST_NAMES[cost], None, ref.params.block_mult,
                                          ref.params.bit_mult)
                chk.insert(keys)
                assert np.array_equal(want, chk.words), f"call {i}: differs from the oracle"
        finally:
            ref.close()
            na.close()


def test_calls_on_top_of_a_filter(dev):
    """A second no-alloc call continues a filter the first one built, as the
    allocating insert does."""
    M, c, k = 1 << 14, 2, 14
    ref, na = pair(M, c, k, "la", seed=5)
    try:
        a = workload.positive_keys(5, (1 << 17) + 3)
        b = workload.negative_keys(5, len(a), (1 << 16) + 1)
        for part in (a, b):
            kd = torch.from_numpy(part.view(np.int64)).to(dev)
            ref.insert_deterministic(kd)
            na.insert_deterministic_noalloc(kd)
        torch.cuda.synchronize()
        assert np.array_equal(na.download(), ref.download())
    finally:
        ref.close()
        na.close()
