"""The synthetic input generators (CPU): planted repeats for the large
genome workload. They hold no filter arithmetic."""

import numpy as np
import pytest

import workload


@pytest.mark.parametrize("n,frac", [(100_000, 0.1), (1_000_000, 0.1), (50_000, 0.3), (10_000, 0.0)])
def test_repeat_segments_cover_without_overlap(n, frac):
    dst, lens, src = workload.repeat_segments(7, n, frac)
    assert len(dst) == len(lens) == len(src)
    if frac == 0:
        assert len(dst) == 0
        return
    assert lens.sum() >= int(frac * n)
    assert lens.sum() < int(frac * n) + 6000
    assert np.all(lens[:-1] >= 300) and np.all(lens <= 6000)
    assert np.all(dst[1:] >= dst[:-1] + lens[:-1]), "segments overlap"
    assert int(dst[-1] + lens[-1]) <= n
    assert np.all(src + lens <= n)


def test_plant_copies_with_divergence():
    n = 400_000
    bases = workload.random_bases(1, n)
    segs = workload.repeat_segments(2, n, 0.2)
    out = workload.plant_numpy(bases, segs, 0.02, 3)
    outside = np.ones(n, dtype=bool)
    diffs, total = 0, 0
    for d, L, s in zip(*segs):
        d, L, s = int(d), int(L), int(s)
        outside[d:d + L] = False
        diffs += int((out[d:d + L] != bases[s:s + L]).sum())
        total += L
    assert np.array_equal(out[outside], bases[outside])
    assert abs(diffs / total - 0.02) < 0.003
