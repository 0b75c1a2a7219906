"""Sequential CPU oracle for Blocked Bloom filters with choices.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark are the only users. The product library never
imports this package, and this package imports nothing from the product.

``bbfc_oracle.c`` holds the definitions (built into ``liboracle.so`` with
gcc); this module is a ctypes wrapper over numpy arrays. ``brute`` is an
independent pure-Python restatement for tiny inputs and ``closed_form``
holds the paper's analytic formulas.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bbfc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

COST_NONE, COST_MIX, COST_LA, COST_EXP = 0, 1, 2, 3
COST_NAMES = {"none": COST_NONE, "mix": COST_MIX, "la": COST_LA, "exp": COST_EXP}


# A sanitizer build (build(sanitize=True)) is loaded instead of liboracle.so
# when this variable names it; the process must then preload gcc's libasan.
LIB_ENV = "BBFC_ORACLE_LIB"


def build(sanitize: bool = False, out: str | None = None) -> str:
    """Compile the oracle with gcc (plain C, no contraction of a*b+c). With
    sanitize=True: AddressSanitizer and UndefinedBehaviorSanitizer, every
    finding fatal, into `out` (default liboracle_san.so beside the source)."""
    out = out or (os.path.join(HERE, "liboracle_san.so") if sanitize else LIB)
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
        "-Wall", "-Wextra", *(san if sanitize else []), "-o", out + ".tmp", SRC, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None
_u64p = ctypes.POINTER(ctypes.c_uint64)


class _Layout(ctypes.Structure):
    """M blocks in T sub-arrays; h_0 has multiplier sub_mult (Section 3.4)."""
    _fields_ = [("M", ctypes.c_uint64), ("T", ctypes.c_uint64), ("sub_mult", ctypes.c_uint64)]


_Lp = ctypes.POINTER(_Layout)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get(LIB_ENV)
    if not path:
        path = LIB
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
    lib = ctypes.CDLL(path)
    u64, u32, i32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
    lib.bbo_hash.argtypes = [u64, u64, u64]
    lib.bbo_hash.restype = u64
    lib.bbo_mask.argtypes = [_u64p, u32, u64, _u64p]
    lib.bbo_mask.restype = None
    lib.bbo_default_param.argtypes = [i32, u32]
    lib.bbo_default_param.restype = dbl
    lib.bbo_cost.argtypes = [i32, dbl, u32, u32, u32]
    lib.bbo_cost.restype = dbl
    lib.bbo_block.argtypes = [_Lp, u64, u64]
    lib.bbo_block.restype = u64
    lib.bbo_insert_one.argtypes = [_u64p, _Lp, u32, u32, i32, i32, dbl, _u64p, _u64p, u64]
    lib.bbo_insert_one.restype = i32
    lib.bbo_insert.argtypes = [_u64p, _Lp, u32, u32, i32, i32, dbl, _u64p, _u64p, _u64p, u64]
    lib.bbo_insert.restype = u64
    lib.bbo_query_one.argtypes = [_u64p, _Lp, u32, u32, i32, _u64p, _u64p, u64]
    lib.bbo_query_one.restype = i32
    lib.bbo_query.argtypes = [_u64p, _Lp, u32, u32, i32, _u64p, _u64p, _u64p, u64, _u64p]
    lib.bbo_query.restype = u64
    lib.bbo_derive_multipliers.argtypes = [u64, u64, u64, u32, u32, i32, _u64p, _u64p, _u64p]
    lib.bbo_derive_multipliers.restype = None
    lib.bbo_envelope.argtypes = [_u64p, _Lp, u32, u32, i32, _u64p, _u64p, _u64p, u64]
    lib.bbo_envelope.restype = None
    lib.bbo_place.argtypes = [_u64p, _Lp, u32, u32, i32, _u64p, _u64p, _u64p, ctypes.c_void_p, u64, u64, u64]
    lib.bbo_place.restype = u64
    lib.bbo_block_loads.argtypes = [_u64p, u64, _u64p]
    lib.bbo_block_loads.restype = None
    lib.bbo_conditional_fpr.argtypes = [_u64p, _Lp, u32, u32, i32, _u64p, _u64p, u64]
    lib.bbo_conditional_fpr.restype = dbl
    lib.bbo_distinct_positions.argtypes = [ctypes.c_void_p, u32, ctypes.c_void_p]
    lib.bbo_distinct_positions.restype = None
    lib.bbo_mask_distinct.argtypes = [_u64p, u32, u64, _u64p]
    lib.bbo_mask_distinct.restype = None
    lib.bbo_qgrams.argtypes = [ctypes.c_void_p, u64, u64, u32, _u64p]
    lib.bbo_qgrams.restype = u64
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def _u64(seq) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(seq, dtype=np.uint64))


def hash_(a: int, x: int, b: int) -> int:
    return int(_load().bbo_hash(a, x, b))


def mask(bit_mult, x: int, distinct: bool = False) -> np.ndarray:
    am = _u64(bit_mult)
    out = np.zeros(8, dtype=np.uint64)
    fn = _load().bbo_mask_distinct if distinct else _load().bbo_mask
    fn(_ptr(am), len(am), x, _ptr(out))
    return out


def distinct_positions(raw) -> list[int]:
    """App. B procedure on raw values (raw[i] in [512 - i])."""
    r = np.ascontiguousarray(raw, dtype=np.uint32)
    out = np.zeros(max(1, len(r)), dtype=np.uint32)
    _load().bbo_distinct_positions(r.ctypes.data, len(r), out.ctypes.data)
    return [int(v) for v in out[:len(r)]]


def default_param(kind: int, k: int) -> float:
    return float(_load().bbo_default_param(kind, k))


def cost(kind: int, param: float, k: int, j: int, a: int) -> float:
    return float(_load().bbo_cost(kind, param, k, j, a))


def qgrams(bases, n_segments: int, seg_len: int, q: int) -> np.ndarray:
    """Canonical q-grams of a base sequence (uint8 values 0..3 = A, C, G, T)."""
    b = np.ascontiguousarray(bases, dtype=np.uint8)
    assert len(b) >= n_segments * seg_len
    n = n_segments * max(0, seg_len - q + 1) if 1 <= q <= 32 else 0
    out = np.zeros(max(1, n), dtype=np.uint64)
    got = _load().bbo_qgrams(b.ctypes.data, n_segments, seg_len, q, _ptr(out))
    assert got == n
    return out[:n]


def derive_multipliers(seed: int, M: int, c: int, k: int, distinct: bool = False, subarrays: int = 1,
                       with_sub: bool = False):
    """Default (block, bit) multipliers; with_sub=True adds the h_0 multiplier."""
    bm = np.zeros(c, dtype=np.uint64)
    am = np.zeros(k, dtype=np.uint64)
    sm = ctypes.c_uint64(0)
    _load().bbo_derive_multipliers(seed, M, subarrays, c, k, int(distinct), _ptr(bm), _ptr(am),
                                   ctypes.cast(ctypes.byref(sm), _u64p))
    out = ([int(v) for v in bm], [int(v) for v in am])
    return out + (int(sm.value),) if with_sub else out


def block_index(n_blocks: int, subarrays: int, sub_mult: int, a: int, x: int) -> int:
    """Candidate block of multiplier a for key x under a sub-array layout."""
    L = _Layout(n_blocks, subarrays, sub_mult)
    return int(_load().bbo_block(ctypes.byref(L), a, x))


class OracleFilter:
    """A filter held in host memory and driven by the sequential oracle."""

    def __init__(self, n_blocks: int, choices: int, k: int, cost_kind: int = COST_NONE,
                 cost_param: float | None = None, block_mult=None, bit_mult=None, seed: int = 0,
                 distinct: bool = False, subarrays: int = 1, sub_mult=None):
        if choices < 1 or k < 1 or n_blocks < 1 or subarrays < 1 or n_blocks % subarrays:
            raise ValueError("bad filter shape")
        self.M, self.c, self.k = int(n_blocks), int(choices), int(k)
        self.T = int(subarrays)
        self.distinct = int(bool(distinct))
        self.kind = int(cost_kind)
        if cost_param is None or (isinstance(cost_param, float) and np.isnan(cost_param)):
            cost_param = default_param(self.kind, self.k)
        self.param = float(cost_param)
        dbm, dam, dsm = derive_multipliers(seed, self.M, self.c, self.k, bool(self.distinct), self.T,
                                           with_sub=True)
        block_mult = dbm if block_mult is None else block_mult
        bit_mult = dam if bit_mult is None else bit_mult
        self.sub_mult = int(dsm if sub_mult is None else sub_mult)
        self.layout = _Layout(self.M, self.T, self.sub_mult)
        self.block_mult = _u64(block_mult)
        self.bit_mult = _u64(bit_mult)
        assert len(self.block_mult) == self.c and len(self.bit_mult) == self.k
        self.words = np.zeros(8 * self.M, dtype=np.uint64)

    def insert(self, keys) -> int:
        keys = _u64(keys)
        return int(_load().bbo_insert(_ptr(self.words), ctypes.byref(self.layout), self.c, self.k, self.distinct, self.kind, self.param,
                                      _ptr(self.block_mult), _ptr(self.bit_mult), _ptr(keys), len(keys)))

    def insert_one(self, key: int) -> int:
        return int(_load().bbo_insert_one(_ptr(self.words), ctypes.byref(self.layout), self.c, self.k, self.distinct, self.kind,
                                          self.param, _ptr(self.block_mult), _ptr(self.bit_mult), key))

    def query_bits(self, keys) -> np.ndarray:
        """Packed answers: bit t of word t//64 (LSB first) for keys[t]."""
        keys = _u64(keys)
        out = np.zeros((len(keys) + 63) // 64, dtype=np.uint64)
        _load().bbo_query(_ptr(self.words), ctypes.byref(self.layout), self.c, self.k, self.distinct, _ptr(self.block_mult),
                          _ptr(self.bit_mult), _ptr(keys), len(keys), _ptr(out))
        return out

    def query(self, keys) -> np.ndarray:
        """Answers as a bool array."""
        bits = self.query_bits(keys)
        n = len(keys)
        return np.unpackbits(bits.view(np.uint8), bitorder="little")[:n].astype(bool)

    def count_hits(self, keys) -> int:
        keys = _u64(keys)
        return int(_load().bbo_query(_ptr(self.words), ctypes.byref(self.layout), self.c, self.k, self.distinct, _ptr(self.block_mult),
                                     _ptr(self.bit_mult), _ptr(keys), len(keys), None))

    def query_one(self, key: int) -> bool:
        return bool(_load().bbo_query_one(_ptr(self.words), ctypes.byref(self.layout), self.c, self.k, self.distinct,
                                          _ptr(self.block_mult), _ptr(self.bit_mult), key))

    def envelope(self, keys) -> np.ndarray:
        keys = _u64(keys)
        env = np.zeros_like(self.words)
        _load().bbo_envelope(_ptr(env), ctypes.byref(self.layout), self.c, self.k, self.distinct, _ptr(self.block_mult),
                             _ptr(self.bit_mult), _ptr(keys), len(keys))
        return env

    def place(self, keys, decisions, words: np.ndarray | None = None, part_mod: int = 1,
              part_rem: int = 0) -> np.ndarray:
        """Words after placing F(keys[t]) in candidate decisions[t] (< c) for
        every key that wrote (decisions[t] >= c: none), on top of `words`
        (default: an empty filter). Only blocks b with b % part_mod ==
        part_rem are written."""
        keys = _u64(keys)
        dec = np.ascontiguousarray(decisions, dtype=np.uint8)
        assert len(dec) == len(keys) and part_mod >= 1 and 0 <= part_rem < part_mod
        out = np.zeros_like(self.words) if words is None else _u64(words).copy()
        _load().bbo_place(_ptr(out), ctypes.byref(self.layout), self.c, self.k, self.distinct,
                          _ptr(self.block_mult), _ptr(self.bit_mult), _ptr(keys), dec.ctypes.data, len(keys),
                          part_mod, part_rem)
        return out

    def insert_recording(self, keys) -> np.ndarray:
        """Sequential insert of keys in order, returning each key's decision:
        the chosen candidate index, or 0xFF when the key was already present."""
        keys = _u64(keys)
        dec = np.empty(len(keys), dtype=np.uint8)
        for t, x in enumerate(keys):
            r = self.insert_one(int(x))
            dec[t] = 0xFF if r < 0 else r
        return dec

    def block_loads(self, words: np.ndarray | None = None) -> np.ndarray:
        w = self.words if words is None else _u64(words)
        hist = np.zeros(513, dtype=np.uint64)
        _load().bbo_block_loads(_ptr(w), self.M, _ptr(hist))
        return hist

    def conditional_fpr(self, keys, words: np.ndarray | None = None) -> float:
        w = self.words if words is None else _u64(words)
        keys = _u64(keys)
        return float(_load().bbo_conditional_fpr(_ptr(w), ctypes.byref(self.layout), self.c, self.k, self.distinct,
                                                 _ptr(self.block_mult), _ptr(keys), len(keys)))
