"""Load histograms and overload on the GPU against the oracle (GPU only).

* the device load histogram (blocks per popcount) equals the oracle's
  count on the same words, for every hash case of M and the extremes;
* App. C, per-block load figure: for k = 7 and 14 and each cost, the GPU's
  racing build has the load distribution of the oracle's sequential build
  (mean, spread, total variation), and more choices give a lower and more
  balanced load, as the paper observes;
* Section 4.1 (overloaded filters) and Section 2.1: inserting gamma times
  the keys a filter was sized for, the GPU build's false-positive rate
  follows the oracle's at every gamma, and grows smoothly with gamma.
"""

import math

import numpy as np
import pytest

import oracle
import paper_2501_18977_amd as bbfc
import workload
from oracle import closed_form as cf

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


def gpu_hist(f):
    h = f.load_histogram()
    torch.cuda.synchronize()
    return h.cpu().numpy().astype(np.uint64)


def moments(h):
    h = np.asarray(h, dtype=np.float64)
    j = np.arange(len(h))
    mean = (h * j).sum() / h.sum()
    sd = math.sqrt((h * (j - mean) ** 2).sum() / h.sum())
    return mean, sd


@pytest.mark.parametrize("M", [1, 7, 3001, 1 << 16, (1 << 16) + 6])
def test_load_histogram_matches_oracle(dev, M):
    bm = workload.draw_multipliers(M, 2, coprime_to=M)
    am = workload.draw_multipliers(M + 1, 11)
    ref = oracle.OracleFilter(M, 2, 11, oracle.COST_EXP, None, bm, am)
    f = bbfc.Filter(M, 2, 11, "exp", block_mult=bm, bit_mult=am)
    try:
        h0 = gpu_hist(f)
        assert h0[0] == M and h0[1:].sum() == 0
        ref.insert(workload.positive_keys(M, max(1, M * 512 // 16)))
        f.upload(ref.words)
        h = gpu_hist(f)
        assert np.array_equal(h, ref.block_loads())
        f.upload(np.full(8 * M, 2**64 - 1, dtype=np.uint64))
        h = gpu_hist(f)
        assert h[512] == M and h[:512].sum() == 0
    finally:
        f.close()


@pytest.mark.parametrize("k", [7, 14])
@pytest.mark.parametrize("cost", ["mix", "la", "exp"])
def test_load_histograms_follow_the_paper(dev, k, cost):
    """Default parameters are the figure's: sigma 2.5 (k = 7) / 50 (k = 14),
    mu 3.5, beta the golden ratio; filter at the standard Bloom size.

    The racing build is one more random build, so the bounds are set by
    sampling noise: two sequential builds with independent multipliers
    differ in total variation by about 0.05 at 2^18 keys (k = 7, EXP) and
    0.026 at 2^20, hence 2^20 keys and a bound of 0.06."""
    n = 1 << 20
    M = math.ceil(n * k / math.log(2) / 512)
    keys = workload.positive_keys(3, n)
    kd = to_dev(keys, dev)
    stats = []
    for c in (1, 2, 3):
        kind = "none" if c == 1 else cost
        bm = workload.draw_multipliers(10 + c, c, coprime_to=M)
        am = workload.draw_multipliers(20 + k, k)
        ref = oracle.OracleFilter(M, c, k, oracle.COST_NAMES[kind], None, bm, am)
        ref.insert(keys)
        f = bbfc.Filter(M, c, k, kind, block_mult=bm, bit_mult=am)
        try:
            f.insert(kd)
            h = gpu_hist(f)
        finally:
            f.close()
        want = ref.block_loads()
        assert h.sum() == M
        gm, gs = moments(h)
        wm, ws = moments(want)
        tv = 0.5 * np.abs(h.astype(np.float64) - want.astype(np.float64)).sum() / M
        print(f"k={k} {cost} c={c}: GPU mean {gm:.2f} sd {gs:.2f}; oracle mean {wm:.2f} sd {ws:.2f}; TV {tv:.3f}",
              flush=True)
        if c == 1:
            assert np.array_equal(h, want)  # one choice: the racing build is the sequential one
        else:
            assert abs(gm - wm) < 0.3
            assert gs == pytest.approx(ws, rel=0.06)
            assert tv < 0.06
        stats.append((gm, gs))
    (m1, s1), (m2, s2), (m3, s3) = stats
    assert m3 < m2 < m1 and s3 < s2 < s1


@pytest.mark.parametrize("c,cost", [(1, "none"), (2, "exp"), (3, "exp"), (2, "mix")])
def test_overload_sweep(dev, c, cost):
    n, k = 1 << 19, 10
    M = math.ceil(n * k / math.log(2) / 512)
    neg = workload.negative_keys(9, 4 * n, 1 << 19)
    bm = workload.draw_multipliers(9, c, coprime_to=M)
    am = workload.draw_multipliers(10, k)
    got_fpr = []
    for gamma in (1.0, 1.1, 1.25, 1.5):
        keys = workload.positive_keys(9, int(gamma * n))
        ref = oracle.OracleFilter(M, c, k, oracle.COST_NAMES[cost], None, bm, am)
        ref.insert(keys)
        f = bbfc.Filter(M, c, k, cost, block_mult=bm, bit_mult=am)
        try:
            f.insert(to_dev(keys, dev))
            words = f.download()
        finally:
            f.close()
        want = ref.conditional_fpr(neg)
        got = ref.conditional_fpr(neg, words=words)
        print(f"c={c} {cost} gamma={gamma}: GPU FPR*2^10 {got * 1024:.3f}, oracle {want * 1024:.3f}", flush=True)
        if c == 1:
            assert np.array_equal(words, ref.words)
            assert got == pytest.approx(cf.blocked_fpr(len(keys), M, k), rel=0.03)
        else:
            assert got == pytest.approx(want, rel=0.02)
        got_fpr.append(got)
    assert all(a < b for a, b in zip(got_fpr, got_fpr[1:]))
    # 10% overload: about the factor 1.912 of a standard Bloom filter (Section 2.1)
    assert 1.5 < got_fpr[1] / got_fpr[0] < 2.2
