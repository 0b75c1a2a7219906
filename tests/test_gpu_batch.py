"""Batched persistent kernels, graphs and the autotuner against the oracle
(GPU only).

* batch query: every filter's answers bit-exact with the oracle's, for all
  launch shapes (lanes per key, tiles per wavefront, occupancy cap);
* batch insert: per filter zero false negatives and every bit inside the
  envelope; bit-exact for one-choice filters; FPR of the larger filters
  within 2% of the oracle's sequential build;
* graphs: every replay equals the eager result, with eager work and
  synchronisations between replays;
* autotuner: returns a valid shape and leaves the filters unchanged.
"""

import itertools
import math

import numpy as np
import pytest

import oracle
import paper_2501_18977_amd as bbfc
import workload

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

COSTS = {"none": oracle.COST_NONE, "mix": oracle.COST_MIX, "la": oracle.COST_LA, "exp": oracle.COST_EXP}
SHAPES = list(itertools.product([8, 4], [1, 2], [0, 2], [0, 3]))


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


# (n keys, space bits per key, k): sizes from empty and one key to 10^5,
# every hash case of M.
SPECS = [(0, 16, 11), (1, 16, 11), (63, 12, 8), (64, 10, 7), (65, 16, 11), (1000, 14, 10),
         (3000, 12, 8), (20000, 16, 11), (100_000, 14, 10), (2, 16, 11), (7000, 10, 7), (65536, 16, 11)]


def build_set(c, cost, seed, dev, specs=SPECS):
    refs, gpus, ns = [], [], []
    for i, (n, bits, k) in enumerate(specs):
        M = max(1, math.ceil(n * bits / 512)) if n else 3
        if i == 9:
            M = 1  # one block
        bm = workload.draw_multipliers(seed + 17 * i, c, coprime_to=M)
        am = workload.draw_multipliers(seed + 17 * i + 5, k)
        refs.append(oracle.OracleFilter(M, c, k, COSTS[cost], None, bm, am))
        gpus.append(bbfc.Filter(M, c, k, cost, block_mult=bm, bit_mult=am))
        ns.append(n)
    return refs, gpus, ns


def keys_for(ns, seed, negatives=False):
    parts = []
    for i, n in enumerate(ns):
        pos = workload.positive_keys(seed + i, n)
        parts.append(np.concatenate([pos, workload.negative_keys(seed + i, n, n)]) if negatives else pos)
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)


def split_answers(out_words, counts):
    res, wo = [], 0
    for n in counts:
        nw = (n + 63) // 64
        res.append(out_words[wo:wo + nw])
        wo += nw
    return res


@pytest.mark.parametrize("lpk,tpw,occ,grab", SHAPES)
def test_batch_query_matches_oracle_for_every_shape(dev, lpk, tpw, occ, grab):
    refs, gpus, ns = build_set(2, "exp", 11, dev)
    for i, (r, g) in enumerate(zip(refs, gpus)):
        r.insert(workload.positive_keys(11 + i, ns[i]))
        g.upload(r.words)
    qn = [2 * n for n in ns]
    plan = bbfc.Batch(gpus, qn)
    plan.set_shape(bbfc.OP_QUERY, lpk, tpw, occ, grab)
    keys = keys_for(ns, 11, negatives=True)
    out = torch.full((plan.total_out_words + 2,), -1, dtype=torch.int64, device=dev)
    plan.query(to_dev(keys, dev), out=out)
    got = from_dev(out)
    assert np.all(got[plan.total_out_words:] == np.uint64(2**64 - 1)), "wrote past the layout"
    per = split_answers(got, qn)
    off = 0
    for i, r in enumerate(refs):
        want = r.query_bits(keys[off:off + qn[i]])
        off += qn[i]
        assert np.array_equal(per[i], want), f"filter {i}"


@pytest.mark.parametrize("c,cost", [(2, "exp"), (3, "mix"), (1, "none")])
def test_batch_insert_invariants(dev, c, cost):
    refs, gpus, ns = build_set(c, cost, 23, dev)
    plan = bbfc.Batch(gpus, ns)
    keys = keys_for(ns, 23)
    kd = to_dev(keys, dev)
    plan.insert(kd)
    # all inserted keys answer true through the batch query and the plain query
    out = from_dev(plan.query(kd))
    per = split_answers(out, ns)
    off = 0
    for i, (r, g) in enumerate(zip(refs, gpus)):
        ks = keys[off:off + ns[i]]
        off += ns[i]
        assert bbfc.unpack_bits(per[i], ns[i]).all(), f"filter {i}: false negative"
        words = g.download()
        r.insert(ks)
        if c == 1:
            assert np.array_equal(words, r.words), f"filter {i}"
        else:
            env = r.envelope(ks)
            assert not np.any(words & ~env), f"filter {i}: bit outside the envelope"
        if ns[i]:
            plain = from_dev(g.query(to_dev(ks, dev)))
            assert np.array_equal(plain, per[i])


def test_batch_insert_fpr_matches_sequential_build(dev):
    specs = [(1 << 18, 16, 11), (100_000, 12, 8), (1 << 16, 14, 10)]
    refs, gpus, ns = build_set(2, "exp", 31, dev, specs)
    plan = bbfc.Batch(gpus, ns)
    keys = keys_for(ns, 31)
    plan.insert(to_dev(keys, dev))
    torch.cuda.synchronize()
    off = 0
    for i, (r, g) in enumerate(zip(refs, gpus)):
        r.insert(keys[off:off + ns[i]])
        off += ns[i]
        neg = workload.negative_keys(31 + i, ns[i], 1 << 22)
        est_gpu = r.conditional_fpr(neg, words=g.download())
        est_ref = r.conditional_fpr(neg)
        print(f"filter {i}: conditional FPR gpu {est_gpu:.4e} oracle {est_ref:.4e}", flush=True)
        assert abs(est_gpu - est_ref) / est_ref < 0.02


def test_graph_replays_equal_eager(dev):
    refs, gpus, ns = build_set(2, "la", 41, dev)
    for i, (r, g) in enumerate(zip(refs, gpus)):
        r.insert(workload.positive_keys(41 + i, ns[i]))
        g.upload(r.words)
    qn = [2 * n for n in ns]
    plan = bbfc.Batch(gpus, qn)
    keys = to_dev(keys_for(ns, 41, negatives=True), dev)
    eager = from_dev(plan.query(keys)).copy()
    out = torch.zeros(plan.total_out_words, dtype=torch.int64, device=dev)
    graph = bbfc.Graph(query_batch=plan, query_keys=keys, out=out)
    for rep in range(4):
        out.zero_()
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(out), eager), f"replay {rep}"
        # eager work between replays, on the same filters
        plan.set_shape(bbfc.OP_QUERY, 4, 2, 0)
        assert np.array_equal(from_dev(plan.query(keys)), eager)
    graph.close()


def test_graph_insert_then_query(dev):
    """One-choice filters make the racing insert deterministic, so every
    replay of insert + query must reproduce the eager filters and answers."""
    refs, gpus, ns = build_set(1, "none", 53, dev)
    ins = bbfc.Batch(gpus, ns)
    qn = [2 * n for n in ns]
    qry = bbfc.Batch(gpus, qn)
    ik = to_dev(keys_for(ns, 53), dev)
    qk = to_dev(keys_for(ns, 53, negatives=True), dev)
    ins.insert(ik)
    eager_ans = from_dev(qry.query(qk)).copy()
    eager_words = [g.download() for g in gpus]
    out = torch.zeros(qry.total_out_words, dtype=torch.int64, device=dev)
    graph = bbfc.Graph(insert_batch=ins, insert_keys=ik, query_batch=qry, query_keys=qk, out=out)
    for rep in range(3):
        for g in gpus:
            g.clear()
        out.zero_()
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(out), eager_ans), f"replay {rep}"
        for g, w in zip(gpus, eager_words):
            assert np.array_equal(g.download(), w)
    graph.close()


@pytest.mark.parametrize("op", [bbfc.OP_QUERY, bbfc.OP_INSERT])
def test_tuner_picks_a_shape_and_preserves_filters(dev, op):
    refs, gpus, ns = build_set(2, "exp", 61, dev)
    for i, (r, g) in enumerate(zip(refs, gpus)):
        r.insert(workload.positive_keys(61 + i, ns[i]))
        g.upload(r.words)
    before = [g.download() for g in gpus]
    if op == bbfc.OP_QUERY:
        plan = bbfc.Batch(gpus, [2 * n for n in ns])
        keys = to_dev(keys_for(ns, 61, negatives=True), dev)
        out = torch.empty(plan.total_out_words, dtype=torch.int64, device=dev)
        best = plan.tune(op, keys, out, reps=1)
    else:
        plan = bbfc.Batch(gpus, ns)
        keys = to_dev(keys_for(ns, 71), dev)
        best = plan.tune(op, keys, reps=1)
    assert best["lanes_per_key"] in (4, 8) and best["tiles_per_wave"] in (1, 2) and best["ms"] > 0
    assert plan.get_shape(op)["lanes_per_key"] == best["lanes_per_key"]
    for g, w in zip(gpus, before):
        assert np.array_equal(g.download(), w)


def test_batch_rejects_bad_plans(dev):
    a = bbfc.Filter(64, 2, 8, "la", seed=1)
    b = bbfc.Filter(64, 3, 8, "la", seed=1)
    with pytest.raises(bbfc.BBFCError, match="same number of choices"):
        bbfc.Batch([a, b], [10, 10])
    plan = bbfc.Batch([a], [10])
    with pytest.raises(bbfc.BBFCError):
        plan.set_shape(bbfc.OP_QUERY, 5, 1, 0)
    with pytest.raises(bbfc.BBFCError):
        plan.set_shape(7, 8, 1, 0)
