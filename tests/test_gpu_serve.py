"""Continuous-batching query server (GPU only).

Every request's answers must be the same when it is served alone, when it
is served in a mix with many other requests (packed into shared batches,
split across batches, overlapping on several streams), and when the
oracle answers the same keys; for requests from host memory and for
requests whose keys and answers stay in device memory.
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


@pytest.fixture(scope="module")
def served(dev):
    """An oracle-built filter uploaded to the device, and its keys."""
    M, c, k = 1 << 14, 2, 11
    bm = workload.draw_multipliers(5, c, coprime_to=M)
    am = workload.draw_multipliers(6, k)
    ref = oracle.OracleFilter(M, c, k, oracle.COST_LA, None, bm, am)
    n = 1 << 18
    keys = workload.positive_keys(5, n)
    ref.insert(keys)
    f = bbfc.Filter(M, c, k, "la", block_mult=bm, bit_mult=am)
    f.upload(ref.words)
    yield ref, f, keys
    f.close()


SIZES = [1, 2, 63, 64, 65, 127, 1000, 4096, 5000, 70_000, 3, 200_000, 17, 64 * 7, 9999]


def make_requests(keys, sizes, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i, s in enumerate(sizes):
        pos = keys[rng.integers(0, len(keys), size=(s + 1) // 2)]
        neg = workload.negative_keys(5, len(keys) + 1000 * i, s // 2)
        r = np.concatenate([pos, neg])
        rng.shuffle(r)
        reqs.append(r)
    return reqs


def test_results_same_alone_in_mix_and_oracle(served):
    ref, f, keys = served
    reqs = make_requests(keys, SIZES, 1)
    srv = bbfc.Server(f, n_slots=3, max_batch_keys=1 << 16)
    try:
        alone = []
        for r in reqs:
            t = srv.submit(r)
            ans, lat = srv.wait(t)
            assert lat > 0
            alone.append(ans.copy())
        b_alone = srv.stats()["batches"]
        tickets = [srv.submit(r) for r in reqs]  # all in flight together
        mixed = [srv.wait(t)[0].copy() for t in tickets]
        b_mixed = srv.stats()["batches"] - b_alone
    finally:
        srv.close()
    for r, a, m in zip(reqs, alone, mixed):
        want = ref.query_bits(r)
        assert np.array_equal(a, want)
        assert np.array_equal(m, want)
    # in the mix, requests shared batches
    assert b_mixed < b_alone


def _dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(dev)


def _host_words(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64) if hasattr(t, "cpu") else t


def test_device_requests_same_alone_in_mix_and_oracle(served, dev):
    """Requests whose keys and answers live in device memory: alone, all in
    flight together, and interleaved with host requests (batches hold one
    kind), every answer equals the oracle's and the host path's."""
    ref, f, keys = served
    reqs = make_requests(keys, SIZES, 11)
    d_reqs = [_dev(r, dev) for r in reqs]
    torch.cuda.synchronize()
    srv = bbfc.Server(f, n_slots=3, max_batch_keys=1 << 16)
    try:
        alone = []
        for r in d_reqs:
            ans, lat = srv.wait(srv.submit_device(r))
            assert lat > 0
            alone.append(_host_words(ans).copy())
        b_alone = srv.stats()["batches"]
        tickets = [srv.submit_device(r) for r in d_reqs]
        mixed = [_host_words(srv.wait(t)[0]).copy() for t in tickets]
        b_mixed = srv.stats()["batches"] - b_alone
        tickets = [(srv.submit_device(d) if i % 2 else srv.submit(h)) for i, (h, d) in enumerate(zip(reqs, d_reqs))]
        both = [_host_words(srv.wait(t)[0]).copy() for t in tickets]
    finally:
        srv.close()
    for r, a, m, b in zip(reqs, alone, mixed, both):
        want = ref.query_bits(r)
        assert np.array_equal(a, want)
        assert np.array_equal(m, want)
        assert np.array_equal(b, want)
    assert b_mixed < b_alone


def test_device_requests_many_pieces(served, dev):
    """3000 tiny device requests in flight at once: batches close at 1024
    pieces, and every request's answer word is exact (bits past n zero)."""
    ref, f, keys = served
    sizes = [1 + (i * 37) % 64 for i in range(3000)]
    reqs = make_requests(keys, sizes, 12)
    flat = np.concatenate(reqs)
    d_flat = _dev(flat, dev)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    outs = torch.full((len(reqs),), -1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    srv = bbfc.Server(f, n_slots=2, max_batch_keys=1 << 20)
    try:
        tickets = [srv.submit_device(d_flat[int(offs[i]):int(offs[i + 1])], out=outs[i:i + 1])
                   for i in range(len(reqs))]
        for t in tickets:
            srv.wait(t)
        assert srv.stats()["batches"] >= len(reqs) // 1024
    finally:
        srv.close()
    got = outs.cpu().numpy().view(np.uint64)
    for i, r in enumerate(reqs):
        assert got[i] == ref.query_bits(r)[0], i


def test_device_replay_under_tight_admission(served, dev):
    ref, f, keys = served
    sizes = [int(round(2 ** u)) for u in np.random.default_rng(13).uniform(0, 13, size=300)]
    reqs = make_requests(keys, sizes, 13)
    flat = np.concatenate(reqs)
    offs = np.zeros(len(reqs) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reqs])
    arrivals = np.cumsum(np.random.default_rng(14).exponential(20e-6, size=len(reqs)))
    srv = bbfc.Server(f, n_slots=4, max_batch_keys=1 << 14, max_pending_keys=5000)
    try:
        out, oo, lat, wall = srv.replay_device(_dev(flat, dev), offs, arrivals)
    finally:
        srv.close()
    words = out.cpu().numpy().view(np.uint64)
    assert wall > 0 and np.all(lat > 0)
    for i, r in enumerate(reqs):
        assert np.array_equal(words[int(oo[i]):int(oo[i + 1])], ref.query_bits(r)), i


@pytest.mark.parametrize("window", [0, 200])
def test_device_requests_with_and_without_batching_window(served, dev, window):
    """Gathering batches for a window (or never) changes only how requests
    are grouped: every answer equals the oracle's."""
    ref, f, keys = served
    reqs = make_requests(keys, [1, 5000, 64, 70_000, 3, 4097] * 4, 15)
    d_reqs = [_dev(r, dev) for r in reqs]
    torch.cuda.synchronize()
    srv = bbfc.Server(f, n_slots=4, max_batch_keys=1 << 14, batch_window_us=window)
    try:
        tickets = [srv.submit_device(r) for r in d_reqs]
        got = [_host_words(srv.wait(t)[0]).copy() for t in tickets]
    finally:
        srv.close()
    for r, g in zip(reqs, got):
        assert np.array_equal(g, ref.query_bits(r))


def test_device_request_overlapping_output_rejected(served, dev):
    _, f, _ = served
    buf = torch.zeros(4096, dtype=torch.int64, device=dev)
    srv = bbfc.Server(f)
    try:
        with pytest.raises(bbfc.BBFCError, match="overlaps"):
            srv.submit_device(buf[:1000], out=buf[900:1000])
    finally:
        srv.close()


def test_large_requests_split_across_small_batches(served):
    ref, f, keys = served
    reqs = make_requests(keys, [100_000, 3, 50_001, 64], 2)
    srv = bbfc.Server(f, n_slots=2, max_batch_keys=4096)
    try:
        tickets = [srv.submit(r) for r in reqs]
        got = [srv.wait(t)[0].copy() for t in tickets]
        assert srv.stats()["batches"] >= 100_000 // 4096
    finally:
        srv.close()
    for r, g in zip(reqs, got):
        assert np.array_equal(g, ref.query_bits(r))


@pytest.mark.parametrize("poll_us", [0, 20])
def test_concurrent_clients(served, poll_us):
    """Six client threads submit and wait at once against eight slots of
    2048 keys, so one request's pieces are served by several slots in
    parallel; every answer equals the oracle's."""
    import threading

    ref, f, keys = served
    per_client = [make_requests(keys, [5000, 1, 70_000, 64, 333, 20_000, 4097], 10 + i) for i in range(6)]
    got = [[None] * len(r) for r in per_client]
    errors = []
    srv = bbfc.Server(f, n_slots=8, max_batch_keys=2048, poll_us=poll_us)

    def client(i):
        try:
            tickets = [srv.submit(r) for r in per_client[i]]
            for j, t in enumerate(tickets):
                got[i][j] = srv.wait(t)[0].copy()
        except Exception as e:  # reported below, on the main thread
            errors.append(e)

    try:
        threads = [threading.Thread(target=client, args=(i,)) for i in range(len(per_client))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        stats = srv.stats()
    finally:
        srv.close()
    assert not errors, errors
    total = sum(len(r) for reqs in per_client for r in reqs)
    assert stats["completed"] == sum(len(r) for r in per_client)
    assert stats["batched_keys"] >= total
    for reqs, answers in zip(per_client, got):
        for r, a in zip(reqs, answers):
            assert np.array_equal(a, ref.query_bits(r))


def test_zero_length_request(served):
    _, f, _ = served
    srv = bbfc.Server(f)
    try:
        t = srv.submit(np.zeros(0, dtype=np.uint64))
        ans, lat = srv.wait(t)
        assert len(ans) == 0 and lat >= 0
    finally:
        srv.close()


def test_replay_under_tight_admission(served):
    """A Poisson schedule replayed against a server that admits at most 5000
    pending keys: requests wait for admission, all answers stay exact."""
    ref, f, keys = served
    sizes = [int(round(2 ** u)) for u in np.random.default_rng(3).uniform(0, 13, size=300)]
    reqs = make_requests(keys, sizes, 3)
    flat = np.concatenate(reqs)
    offs = np.zeros(len(reqs) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reqs])
    arrivals = np.cumsum(np.random.default_rng(4).exponential(20e-6, size=len(reqs)))
    srv = bbfc.Server(f, n_slots=4, max_batch_keys=1 << 14, max_pending_keys=5000)
    try:
        answers, lat, wall = srv.replay(flat, offs, arrivals)
    finally:
        srv.close()
    assert wall > 0 and np.all(lat > 0)
    for r, a in zip(reqs, answers):
        assert np.array_equal(a, ref.query_bits(r))


def test_server_config_validation(served):
    _, f, _ = served
    for kw in ({"n_slots": 0}, {"n_slots": 17}, {"max_batch_keys": 100}, {"max_pending_keys": 0},
               {"batch_window_us": 100001}):
        with pytest.raises(bbfc.BBFCError):
            bbfc.Server(f, **kw)


def test_wait_unknown_ticket(served):
    _, f, _ = served
    srv = bbfc.Server(f)
    try:
        with pytest.raises(bbfc.BBFCError, match="unknown ticket"):
            srv.wait(12345)
    finally:
        srv.close()


def test_serving_while_inserting(dev):
    """Requests served while an insert into the same filter runs on another
    stream: every served answer is also an answer after the insert (bits are
    only set), and after it every inserted key answers true."""
    M, n = 1 << 16, 1 << 21
    f = bbfc.Filter(M, 2, 11, "la", seed=41)
    srv = bbfc.Server(f, n_slots=4, max_batch_keys=1 << 16)
    try:
        keys_d = workload.device_keys(41, 0, n, device=dev)
        torch.cuda.synchronize()
        host = keys_d.cpu().numpy().view(np.uint64)
        reqs = [host[i * 50_000:(i + 1) * 50_000] for i in range(20)]
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            f.insert(keys_d)
        tickets = [srv.submit(r) for r in reqs]
        during = [srv.wait(t)[0].copy() for t in tickets]
        torch.cuda.synchronize()
        tickets = [srv.submit(r) for r in reqs]
        after = [srv.wait(t)[0].copy() for t in tickets]
    finally:
        srv.close()
        f.close()
    for r, d, a in zip(reqs, during, after):
        assert not np.any(d & ~a)
        assert bbfc.unpack_bits(a, len(r)).all()


def test_close_with_requests_in_flight(served):
    """Closing the server with admitted requests that nobody waited for
    serves them first: their answer buffers are filled when close returns."""
    ref, f, keys = served
    reqs = make_requests(keys, [70_000, 5, 4096, 200_000], 7)
    srv = bbfc.Server(f, n_slots=2, max_batch_keys=1 << 14)
    tickets = [srv.submit(r) for r in reqs]
    outs = [srv._live[t][1] for t in tickets]
    srv.close()
    for r, o in zip(reqs, outs):
        assert np.array_equal(o[: (len(r) + 63) // 64], ref.query_bits(r))
