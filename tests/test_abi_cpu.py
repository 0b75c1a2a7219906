"""The C-ABI library on the CPU: it loads, exports every declared symbol,
and its host-side pieces (hash code shared with the kernels, cost rank
table, argument checks) agree with the oracle. No device call is made."""

import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_2501_18977_amd as bbfc
import workload
from paper_2501_18977_amd import _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if _build.is_stale():
        _build.build()
    return bbfc.lib()


def declared_functions():
    with open(os.path.join(ROOT, "include", "bbfc.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbfc_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    L = bbfc.lib()
    for name in names:
        assert hasattr(L, name), name


def test_no_undeclared_exports_beyond_header():
    out = os.popen(f"nm -D --defined-only {bbfc.library_path()}").read()
    exported = {m for m in re.findall(r" T (bbfc_[a-z0-9_]+)$", out, flags=re.M)}
    assert exported == set(declared_functions())


@pytest.mark.parametrize("M", [1, 2, 8, 1 << 15, 1 << 25, 6, 3_000_000, 3 * (1 << 20), 9, 1001, 79_299_999,
                               (1 << 33) + 1, (1 << 40) + 6, (1 << 63) + 7])
def test_block_hash_source_matches_oracle(M):
    """The kernels' block hash (compiled for the host) equals the oracle's
    for the power-of-two, even and odd cases, including the invariant-
    divisor remainder at large moduli."""
    rng = np.random.default_rng(M % 1000)
    mults = workload.draw_multipliers(M % 97, 8, coprime_to=M)
    keys = list(workload.positive_keys(M % 89, 200)) + [0, 1, (1 << 64) - 1, 1 << 63]
    for a in mults:
        for x in keys:
            x = int(x)
            assert bbfc.host_block_hash(M, a, x) == oracle.hash_(a, x, M)
    for _ in range(200):
        a = int(rng.integers(0, 1 << 63)) * 2 + 1
        x = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        assert bbfc.host_block_hash(M, a, x) == oracle.hash_(a, x, M)


@pytest.mark.parametrize("M,T", [(1 << 15, 1 << 6), (1 << 15, 1), (3 * 1024, 3), (6000, 12), (7, 7),
                                 ((1 << 25), 1 << 15), (1001 * 64, 1001)])
def test_block_index_source_matches_oracle(M, T):
    """Sub-array addressing (Section 3.4, Parallelization) compiled for the
    host: h_0(x) S + h_i(x) equals the oracle's for pow2, even and odd T, S."""
    S = M // T
    sm = workload.draw_multipliers(T, 1, coprime_to=T)[0] if T > 1 else 0
    for a in workload.draw_multipliers(M % 91, 3, coprime_to=S):
        for x in list(workload.positive_keys(M % 53, 300)) + [0, (1 << 64) - 1]:
            assert bbfc.host_block_index(M, T, sm, a, int(x)) == oracle.block_index(M, T, sm, a, int(x))


def test_bit_hash_source_matches_oracle():
    for a in workload.draw_multipliers(3, 16):
        for x in workload.positive_keys(3, 300):
            assert bbfc.host_bit_hash(a, int(x)) == oracle.hash_(a, int(x), 512)


@pytest.mark.parametrize("kind", [bbfc.COST_MIX, bbfc.COST_LA, bbfc.COST_EXP])
@pytest.mark.parametrize("k", [1, 2, 7, 8, 10, 11, 14, 20, 32])
def test_rank_table_orders_pairs_like_oracle_costs(kind, k):
    """For all feasible (j, a) pairs, rank(p) < rank(q) iff cost(p) < cost(q)
    with the oracle's double costs, and equal ranks iff equal doubles."""
    table = bbfc.rank_table(kind, k)
    par = oracle.default_param(kind, k)
    pairs, costs, ranks = [], [], []
    for a in range(1, k + 1):
        for j in range(a, 513):
            pairs.append((j, a))
            costs.append(oracle.cost(kind, par, k, j, a))
            ranks.append(int(table[a, j]))
    costs = np.array(costs)
    ranks = np.array(ranks)
    order = np.argsort(costs, kind="stable")
    c_sorted, r_sorted = costs[order], ranks[order]
    same = c_sorted[1:] == c_sorted[:-1]
    assert np.all(r_sorted[1:][same] == r_sorted[:-1][same])
    assert np.all(r_sorted[1:][~same] > r_sorted[:-1][~same])
    assert np.all(table[0] == 0xFFFF)
    for a in range(1, k + 1):
        assert np.all(table[a, :a] == 0xFFFF)


def test_rank_table_explicit_param():
    t1 = bbfc.rank_table("mix", 14, 50.0)
    t2 = bbfc.rank_table("mix", 14)
    assert np.array_equal(t1, t2)
    t3 = bbfc.rank_table("mix", 14, 2.5)
    assert not np.array_equal(t1, t3)


def test_blocks_for():
    assert bbfc.blocks_for(1 << 20, 16) == 1 << 15
    assert bbfc.blocks_for(1 << 30, 16) == 1 << 25
    assert bbfc.blocks_for(1000, 12) == math.ceil(1000 * 12 / 512)
    assert bbfc.blocks_for(0, 12) == 1
    assert bbfc.blocks_for(1, 1) == 1


def test_status_strings():
    L = bbfc.lib()
    for s in (0, -1, -2, -3, -4, -99):
        assert L.bbfc_status_string(s)


@pytest.mark.parametrize("args,needle", [
    ((0, 2, 8, "la"), "n_blocks"),
    ((64, 0, 8, "la"), "choices"),
    ((64, 5, 8, "la"), "choices"),
    ((64, 2, 0, "la"), "bits_per_key"),
    ((64, 2, 33, "la"), "bits_per_key"),
    ((64, 1, 8, "la"), "one choice"),
    ((64, 2, 8, "none"), "cost kind"),
])
def test_create_rejects_bad_shapes_before_touching_the_device(args, needle):
    with pytest.raises(bbfc.BBFCError) as e:
        bbfc.Filter(*args)
    assert e.value.status == -1
    assert needle in str(e.value)


def test_create_rejects_bad_multipliers():
    with pytest.raises(bbfc.BBFCError, match="coprime"):
        bbfc.Filter(6, 2, 4, "exp", block_mult=[3 | (1 << 40), 5 | (1 << 40)], bit_mult=[(1 << 40) + 1] * 4)
    with pytest.raises(bbfc.BBFCError, match="bit multiplier 1 is not coprime to its modulus 512"):
        bbfc.Filter(8, 2, 2, "exp", block_mult=[(1 << 40) + 1] * 2, bit_mult=[(1 << 40) + 1, 1 << 40])
    # distinct selection: bit hash 1 reduces modulo 511 = 7 * 73
    with pytest.raises(bbfc.BBFCError, match="bit multiplier 1 is not coprime to its modulus 511"):
        bbfc.Filter(8, 2, 2, "exp", block_mult=[(1 << 40) + 1] * 2, bit_mult=[(1 << 40) + 1, 7 * ((1 << 40) + 1)],
                    bit_selection="distinct")
    with pytest.raises(bbfc.BBFCError, match="unknown bit selection"):
        bbfc.Filter(8, 2, 2, "exp", bit_selection=5)
    with pytest.raises(bbfc.BBFCError, match="must divide n_blocks"):
        bbfc.Filter(1000, 2, 8, "exp", subarrays=3)
    with pytest.raises(bbfc.BBFCError, match="not coprime to subarrays"):
        bbfc.Filter(1024, 2, 8, "exp", subarrays=4, sub_mult=(1 << 40) + 2)
    with pytest.raises(bbfc.BBFCError, match="blocks per sub-array"):
        bbfc.Filter(3 * 512, 2, 8, "exp", subarrays=512, block_mult=[3 * ((1 << 40) + 1)] * 2,
                    bit_mult=[(1 << 40) + 1] * 8)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 14, 17, 20, 31, 32])
@pytest.mark.parametrize("sel", ["random", "distinct"])
def test_key_mask_source_matches_oracle(k, sel):
    """The kernels' bit selection code (compiled for the host) gives the
    oracle's F(x), for both strategies (Section 3.3, App. B). The device
    computes distinct addresses by counting free addresses, the oracle by
    the paper's insertion sort: they share nothing but the definition."""
    distinct = sel == "distinct"
    am = workload.draw_multipliers(k + 7, k, coprime_to=workload.distinct_moduli(k) if distinct else 512)
    keys = list(workload.positive_keys(k, 3000)) + [0, 1, (1 << 64) - 1]
    for x in keys:
        got = bbfc.host_key_mask(am, int(x), sel)
        want = oracle.mask(am, int(x), distinct=distinct)
        assert np.array_equal(got, want), (k, sel, int(x))


def test_key_mask_argument_errors():
    with pytest.raises(bbfc.BBFCError):
        bbfc.host_key_mask([], 1)
    with pytest.raises(bbfc.BBFCError):
        bbfc.host_key_mask([(1 << 40) + 1] * 33, 1)
    with pytest.raises(bbfc.BBFCError):
        bbfc.host_key_mask([(1 << 40) + 1], 1, 2)


def test_null_handle_calls_are_rejected():
    L = bbfc.lib()
    assert L.bbfc_insert(None, None, 0, None) == -1
    assert L.bbfc_query(None, None, 0, None, None) == -1
    assert L.bbfc_destroy(None) == -1
    assert L.bbfc_clear(None, None) == -1


def test_server_default_config():
    """The defaults that a null server config stands for (host-only call)."""
    import ctypes

    cfg = bbfc._ServerConfig()
    assert bbfc.lib().bbfc_server_default_config(ctypes.byref(cfg)) == 0
    assert (cfg.n_slots, cfg.max_batch_keys, cfg.max_pending_keys, cfg.poll_us, cfg.batch_window_us) == \
        (4, 1 << 20, 1 << 28, 20, 0)
    assert bbfc.lib().bbfc_server_default_config(None) == -1


def test_workload_generators_agree():
    keys = workload.splitmix64_keys(123, 1000, 64)
    for i, v in enumerate(keys):
        assert int(v) == workload.splitmix64_scalar(123, 1000 + i)
    assert len(set(workload.positive_keys(0, 5000)) & set(workload.negative_keys(0, 5000, 5000))) == 0


def test_missing_library_fails_loudly():
    """Without the built HIP library the binding raises; there is no CPU path."""
    import subprocess
    import sys

    code = (
        "import paper_2501_18977_amd as bbfc\n"
        "bbfc._LIB_PATH = '/nonexistent/libbbfc.so'\n"
        "try:\n"
        "    bbfc.Filter(1024, 2, 8, 'la', seed=1)\n"
        "except RuntimeError as e:\n"
        "    assert 'no fallback' in str(e), e\n"
        "    print('raised')\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "raised"
