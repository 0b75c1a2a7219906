"""Blocked Bloom filters with choices on AMD MI355X (gfx950).

Python binding of the C ABI in ``include/bbfc.h``: argument marshalling only.
Every insert and query runs in the HIP kernels of ``libbbfc.so``; there is no
CPU fallback, and a missing library raises an error.

Keys are 64-bit CUDA/HIP tensors (``torch.int64`` or ``torch.uint64``; the bits
are what count). Work is enqueued on the current torch stream unless a
stream is given.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "BBFCError",
    "COST_NONE",
    "COST_MIX",
    "COST_LA",
    "COST_EXP",
    "Filter",
    "Batch",
    "Graph",
    "Server",
    "blocks_for",
    "rank_table",
    "host_block_hash",
    "kmer_count",
    "kmer_keys",
    "host_bit_hash",
    "host_key_mask",
    "host_block_index",
    "lib",
    "library_path",
    "probe_gather",
    "probe_atomic64",
    "probe_copy",
    "probe_insert_schedule",
    "unpack_bits",
]

COST_NONE, COST_MIX, COST_LA, COST_EXP = 0, 1, 2, 3
BITS_RANDOM, BITS_DISTINCT = 0, 1
_BITS_BY_NAME = {"random": BITS_RANDOM, "distinct": BITS_DISTINCT}
OP_INSERT, OP_QUERY = 0, 1
OPT_INSERT_INFLIGHT, OPT_QUERY_EARLY_EXIT, OPT_INSERT_TILE = 1, 2, 3
DECISION_PRESENT = 0xFF
_COST_BY_NAME = {"none": COST_NONE, "mix": COST_MIX, "la": COST_LA, "exp": COST_EXP}

_HERE = os.path.dirname(os.path.abspath(__file__))
# BBFC_LIBRARY names another build of the same library to load instead (the
# CPU tests use it for a build whose host code carries sanitizers).
_LIB_PATH = os.environ.get("BBFC_LIBRARY") or os.path.join(_HERE, "libbbfc.so")


class BBFCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bbfc error {status}: {message}")
        self.status = status


class _Cost(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("param", ctypes.c_double)]


class _Config(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_uint64), ("choices", ctypes.c_uint32), ("bits_per_key", ctypes.c_uint32),
                ("cost", _Cost), ("bit_selection", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("block_mult", ctypes.c_void_p), ("bit_mult", ctypes.c_void_p),
                ("subarrays", ctypes.c_uint64), ("sub_mult", ctypes.c_uint64)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_uint32), ("max_batch_keys", ctypes.c_uint64),
                ("max_pending_keys", ctypes.c_uint64), ("poll_us", ctypes.c_uint32),
                ("batch_window_us", ctypes.c_uint32)]


class _Shape(ctypes.Structure):
    _fields_ = [("lanes_per_key", ctypes.c_int32), ("tiles_per_wave", ctypes.c_int32),
                ("wgs_per_cu", ctypes.c_int32), ("units_per_grab", ctypes.c_int32), ("ms", ctypes.c_float)]


_lib = None
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_vp = ctypes.c_void_p
_st = ctypes.c_int


def library_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """The loaded ``libbbfc.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(hipcc --offload-arch=gfx950); there is no fallback path"
        )
    L = ctypes.CDLL(_LIB_PATH)
    sig = {
        "bbfc_create": (_st, [_u64, _u32, _u32, _Cost, _vp]),
        "bbfc_create_seeded": (_st, [_u64, _u32, _u32, _Cost, _u64, _vp]),
        "bbfc_create_with_multipliers": (_st, [_u64, _u32, _u32, _Cost, _vp, _vp, _vp]),
        "bbfc_create_config": (_st, [_vp, _vp]),
        "bbfc_get_bit_selection": (_st, [_vp, _vp]),
        "bbfc_get_subarrays": (_st, [_vp, _vp, _vp]),
        "bbfc_bulk_insert": (_st, [_vp, _vp, _u64, _vp, _u64, _vp]),
        "bbfc_bulk_insert_workspace": (_st, [_vp, _u64, _vp]),
        "bbfc_host_block_index": (_u64, [_u64, _u64, _u64, _u64, _u64]),
        "bbfc_load_histogram": (_st, [_vp, _vp, _vp]),
        "bbfc_host_key_mask": (_st, [_vp, _u32, ctypes.c_int32, _u64, _vp]),
        "bbfc_destroy": (_st, [_vp]),
        "bbfc_insert": (_st, [_vp, _vp, _u64, _vp]),
        "bbfc_insert_deterministic": (_st, [_vp, _vp, _u64, _vp]),
        "bbfc_insert_recorded": (_st, [_vp, _vp, _u64, _vp, _vp]),
        "bbfc_insert_deterministic_noalloc": (_st, [_vp, _vp, _u64, _vp]),
        "bbfc_query": (_st, [_vp, _vp, _u64, _vp, _vp]),
        "bbfc_clear": (_st, [_vp, _vp]),
        "bbfc_upload": (_st, [_vp, _vp, _vp]),
        "bbfc_download": (_st, [_vp, _vp, _vp]),
        "bbfc_get_params": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "bbfc_get_words": (_st, [_vp, _vp]),
        "bbfc_set_option": (_st, [_vp, ctypes.c_int32, ctypes.c_int64]),
        "bbfc_get_option": (_st, [_vp, ctypes.c_int32, _vp]),
        "bbfc_server_default_config": (_st, [_vp]),
        "bbfc_insert_launch_info": (_st, [_vp, ctypes.c_uint64, _vp, _vp, _vp]),
        "bbfc_blocks_for": (_u64, [_u64, ctypes.c_double]),
        "bbfc_rank_table": (_st, [_Cost, _u32, _vp]),
        "bbfc_status_string": (ctypes.c_char_p, [_st]),
        "bbfc_last_error": (ctypes.c_char_p, []),
        "bbfc_probe_gather": (_st, [_vp, _u64, _u32, _u64, _u64, _vp, _vp]),
        "bbfc_probe_atomic64": (_st, [_vp, _u64, _u64, _u64, _vp]),
        "bbfc_probe_copy": (_st, [_vp, _vp, _u64, _u32, _vp]),
        "bbfc_probe_insert_pattern": (_st, [_vp, _u64, _u64, ctypes.c_int32, _u64, _vp, _vp]),
        "bbfc_probe_insert_schedule": (_st, [_vp, _u64, _u64, ctypes.c_int32, ctypes.c_int32, _u64, _vp, _vp]),
        "bbfc_probe_latency": (_st, [_vp, _u64, ctypes.c_int32, _u32, _u32, _vp, _vp]),
        "bbfc_batch_create": (_st, [_vp, _vp, _u32, _vp]),
        "bbfc_batch_destroy": (_st, [_vp]),
        "bbfc_batch_layout": (_st, [_vp, _vp, _vp]),
        "bbfc_batch_insert": (_st, [_vp, _vp, _vp]),
        "bbfc_batch_query": (_st, [_vp, _vp, _vp, _vp]),
        "bbfc_batch_set_shape": (_st, [_vp, ctypes.c_int32, _Shape]),
        "bbfc_batch_get_shape": (_st, [_vp, ctypes.c_int32, _vp]),
        "bbfc_batch_tune": (_st, [_vp, ctypes.c_int32, _vp, _vp, _u32, _vp, _vp]),
        "bbfc_set_shape": (_st, [_vp, ctypes.c_int32, _Shape]),
        "bbfc_get_shape": (_st, [_vp, ctypes.c_int32, _vp]),
        "bbfc_tune": (_st, [_vp, ctypes.c_int32, _vp, _u64, _vp, _u32, _vp, _vp]),
        "bbfc_graph_create": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "bbfc_graph_launch": (_st, [_vp, _vp]),
        "bbfc_graph_destroy": (_st, [_vp]),
        "bbfc_server_create": (_st, [_vp, _vp, _vp]),
        "bbfc_server_destroy": (_st, [_vp]),
        "bbfc_server_submit": (_st, [_vp, _vp, _u64, _vp, _vp]),
        "bbfc_server_wait": (_st, [_vp, _u64, ctypes.c_double, _vp]),
        "bbfc_server_stats": (_st, [_vp, _vp, _vp, _vp]),
        "bbfc_server_replay": (_st, [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp]),
        "bbfc_server_submit_device": (_st, [_vp, _vp, _u64, _vp, _vp]),
        "bbfc_server_replay_device": (_st, [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp]),
        "bbfc_kmer_count": (_u64, [_u64, _u64, _u32]),
        "bbfc_kmer_keys": (_st, [_vp, _u64, _u64, _u32, _vp, _vp]),
        "bbfc_insert_kmers": (_st, [_vp, _vp, _u64, _u64, _u32, _vp]),
        "bbfc_query_kmers": (_st, [_vp, _vp, _u64, _u64, _u32, _vp, _vp]),
        "bbfc_host_block_hash": (_u64, [_u64, _u64, _u64]),
        "bbfc_host_bit_hash": (_u32, [_u64, _u64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int) -> None:
    if status != 0:
        msg = lib().bbfc_last_error().decode(errors="replace")
        raise BBFCError(status, msg)


def _cost_struct(cost, param) -> _Cost:
    kind = _COST_BY_NAME[cost] if isinstance(cost, str) else int(cost)
    return _Cost(kind, float("nan") if param is None else float(param))


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _device_u64(t, what: str):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a GPU tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"{what} must be int64 or uint64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


def blocks_for(n_keys: int, space_bits_per_key: float) -> int:
    return int(lib().bbfc_blocks_for(n_keys, space_bits_per_key))


def rank_table(cost, bits_per_key: int, param=None):
    """The cost rank table as a numpy uint16 array of shape (k+1, 513)."""
    import numpy as np

    out = np.empty((bits_per_key + 1) * 513, dtype=np.uint16)
    _check(lib().bbfc_rank_table(_cost_struct(cost, param), bits_per_key, out.ctypes.data))
    return out.reshape(bits_per_key + 1, 513)


def kmer_count(n_segments: int, seg_len: int, q: int) -> int:
    return int(lib().bbfc_kmer_count(n_segments, seg_len, q))


def kmer_keys(seq, n_segments: int, seg_len: int, q: int = 31, out=None, stream=None):
    """The canonical q-grams of a 2-bit packed sequence as an int64 GPU tensor."""
    import torch

    seq = _device_u64(seq, "seq")
    n = kmer_count(n_segments, seg_len, q)
    if out is None:
        out = torch.empty(max(1, n), dtype=torch.int64, device=seq.device)
    _check(lib().bbfc_kmer_keys(seq.data_ptr(), n_segments, seg_len, q, out.data_ptr(), _stream_handle(stream)))
    return out[:n]


def host_block_hash(n_blocks: int, a: int, x: int) -> int:
    return int(lib().bbfc_host_block_hash(n_blocks, a, x))


def host_bit_hash(a: int, x: int) -> int:
    return int(lib().bbfc_host_bit_hash(a, x))


def _bits_id(bit_selection) -> int:
    if isinstance(bit_selection, str):
        return _BITS_BY_NAME[bit_selection]
    return int(bit_selection)


def host_block_index(n_blocks: int, subarrays: int, sub_mult: int, a: int, x: int) -> int:
    return int(lib().bbfc_host_block_index(n_blocks, subarrays, sub_mult, a, x))


def host_key_mask(bit_mult, x: int, bit_selection="random"):
    """F(x) as 8 uint64 words (numpy), computed by the library's host build
    of the kernels' bit selection code."""
    import numpy as np

    am = (ctypes.c_uint64 * len(bit_mult))(*[int(v) for v in bit_mult])
    out = np.zeros(8, dtype=np.uint64)
    _check(lib().bbfc_host_key_mask(am, len(bit_mult), _bits_id(bit_selection), x, out.ctypes.data))
    return out


@dataclass(frozen=True)
class Params:
    n_blocks: int
    choices: int
    bits_per_key: int
    cost_kind: int
    cost_param: float
    block_mult: tuple
    bit_mult: tuple
    bit_selection: int = BITS_RANDOM
    subarrays: int = 1
    sub_mult: int = 0


class Filter:
    """One filter resident in device memory (owned by the library)."""

    def __init__(self, n_blocks: int, choices: int, bits_per_key: int, cost="none", cost_param=None, *,
                 seed: int | None = None, block_mult=None, bit_mult=None, bit_selection="random",
                 subarrays: int = 1, sub_mult: int | None = None):
        L = lib()
        h = ctypes.c_void_p()
        cs = _cost_struct(cost, cost_param)
        sel = _bits_id(bit_selection)
        if sel != BITS_RANDOM or subarrays > 1:
            if block_mult is not None and len(block_mult) != choices:
                raise ValueError("block_mult needs `choices` entries")
            if bit_mult is not None and len(bit_mult) != bits_per_key:
                raise ValueError("bit_mult needs `bits_per_key` entries")
            bm = (ctypes.c_uint64 * choices)(*[int(v) for v in block_mult]) if block_mult is not None else None
            am = (ctypes.c_uint64 * bits_per_key)(*[int(v) for v in bit_mult]) if bit_mult is not None else None
            cfg = _Config(n_blocks, choices, bits_per_key, cs, sel, 0 if seed is None else seed,
                          ctypes.cast(bm, ctypes.c_void_p) if bm is not None else None,
                          ctypes.cast(am, ctypes.c_void_p) if am is not None else None,
                          subarrays, 0 if sub_mult is None else int(sub_mult))
            _check(L.bbfc_create_config(ctypes.byref(cfg), ctypes.byref(h)))
        elif block_mult is not None or bit_mult is not None:
            if block_mult is None or bit_mult is None:
                raise ValueError("give both block_mult and bit_mult")
            bm = (ctypes.c_uint64 * len(block_mult))(*[int(v) for v in block_mult])
            am = (ctypes.c_uint64 * len(bit_mult))(*[int(v) for v in bit_mult])
            if len(block_mult) != choices or len(bit_mult) != bits_per_key:
                raise ValueError("multiplier counts must equal choices and bits_per_key")
            _check(L.bbfc_create_with_multipliers(n_blocks, choices, bits_per_key, cs, bm, am, ctypes.byref(h)))
        elif seed is not None:
            _check(L.bbfc_create_seeded(n_blocks, choices, bits_per_key, cs, seed, ctypes.byref(h)))
        else:
            _check(L.bbfc_create(n_blocks, choices, bits_per_key, cs, ctypes.byref(h)))
        self._h = h
        self.params = self._read_params()

    # -------------------------------------------------------------- info
    def _read_params(self) -> Params:
        M, c, k = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32()
        cs = _Cost()
        bm = (ctypes.c_uint64 * 4)()
        am = (ctypes.c_uint64 * 32)()
        _check(lib().bbfc_get_params(self._h, ctypes.byref(M), ctypes.byref(c), ctypes.byref(k), ctypes.byref(cs),
                                     bm, am))
        sel = ctypes.c_int32()
        _check(lib().bbfc_get_bit_selection(self._h, ctypes.byref(sel)))
        T, sm = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().bbfc_get_subarrays(self._h, ctypes.byref(T), ctypes.byref(sm)))
        return Params(M.value, c.value, k.value, cs.kind, cs.param, tuple(bm[: c.value]), tuple(am[: k.value]),
                      sel.value, T.value, sm.value)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("filter is closed")
        return self._h

    @property
    def n_blocks(self) -> int:
        return self.params.n_blocks

    @property
    def words_ptr(self) -> int:
        p = ctypes.c_void_p()
        _check(lib().bbfc_get_words(self.handle, ctypes.byref(p)))
        return int(p.value)

    def set_option(self, option: int, value: int) -> None:
        _check(lib().bbfc_set_option(self.handle, option, int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64()
        _check(lib().bbfc_get_option(self.handle, option, ctypes.byref(v)))
        return int(v.value)

    def insert_launch_info(self, n: int) -> dict:
        """What an insert of n keys would launch: keys per wavefront tile,
        the keys it works on at once, and workgroups (nothing launched)."""
        tile, inflight, wgs = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().bbfc_insert_launch_info(self.handle, int(n), ctypes.byref(tile), ctypes.byref(inflight),
                                             ctypes.byref(wgs)))
        return {"tile_keys": int(tile.value), "keys_in_flight": int(inflight.value), "workgroups": int(wgs.value)}

    def set_shape(self, op: int, lanes_per_key: int = 8, tiles_per_wave: int = 1, wgs_per_cu: int = 0) -> None:
        _check(lib().bbfc_set_shape(self.handle, op, _Shape(lanes_per_key, tiles_per_wave, wgs_per_cu, 0, 0.0)))

    def get_shape(self, op: int) -> dict:
        sh = _Shape()
        _check(lib().bbfc_get_shape(self.handle, op, ctypes.byref(sh)))
        return _shape_dict(sh)

    def tune(self, op: int, keys, out=None, reps: int = 2, stream=None) -> dict:
        """Time the launch shapes of `op` on these keys and keep the fastest
        (the filter's words are unchanged afterwards)."""
        keys = _device_u64(keys, "keys")
        optr = out.data_ptr() if out is not None else None
        sh = _Shape()
        _check(lib().bbfc_tune(self.handle, op, keys.data_ptr(), keys.numel(), optr, reps, _stream_handle(stream),
                               ctypes.byref(sh)))
        return _shape_dict(sh)

    # -------------------------------------------------------------- ops
    def insert(self, keys, stream=None) -> None:
        """Racing insert (bbfc_insert): at most the filter's bound on keys in
        flight (OPT_INSERT_INFLIGHT; default n_blocks/(8(c-1)), none with one
        choice), in tiles of 8 keys where that bound is small
        (OPT_INSERT_TILE; see insert_launch_info)."""
        keys = _device_u64(keys, "keys")
        _check(lib().bbfc_insert(self.handle, keys.data_ptr(), keys.numel(), _stream_handle(stream)))

    def insert_recorded(self, keys, out=None, stream=None):
        """The racing insert, also returning each key's decision as a uint8
        GPU tensor: the candidate index that received the key's bits, or
        DECISION_PRESENT when a candidate already held them."""
        import torch

        keys = _device_u64(keys, "keys")
        n = keys.numel()
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.uint8, device=keys.device)
        elif out.dtype != torch.uint8 or not out.is_cuda or not out.is_contiguous() or out.numel() < n:
            raise ValueError("decisions need a contiguous uint8 GPU tensor of n entries")
        _check(lib().bbfc_insert_recorded(self.handle, keys.data_ptr(), n, out.data_ptr(), _stream_handle(stream)))
        return out[:n]

    def insert_deterministic(self, keys, stream=None) -> None:
        keys = _device_u64(keys, "keys")
        _check(lib().bbfc_insert_deterministic(self.handle, keys.data_ptr(), keys.numel(), _stream_handle(stream)))

    def insert_deterministic_noalloc(self, keys, stream=None) -> None:
        """insert_deterministic without any device allocation (its scratch is a
        static device array shared by every call on the device)."""
        keys = _device_u64(keys, "keys")
        _check(lib().bbfc_insert_deterministic_noalloc(self.handle, keys.data_ptr(), keys.numel(),
                                                       _stream_handle(stream)))

    def query(self, keys, out=None, stream=None):
        """Packed answers: an int64 tensor of ceil(n/64) words (bit t%64 of
        word t//64 answers keys[t])."""
        import torch

        keys = _device_u64(keys, "keys")
        n = keys.numel()
        n_words = (n + 63) // 64
        if out is None:
            out = torch.empty(max(n_words, 1), dtype=torch.int64, device=keys.device)
        else:
            out = _device_u64(out, "out")
            if out.numel() < n_words:
                raise ValueError("output too small")
        _check(lib().bbfc_query(self.handle, keys.data_ptr(), n, out.data_ptr(), _stream_handle(stream)))
        return out

    def insert_kmers(self, seq, n_segments: int, seg_len: int, q: int = 31, stream=None) -> None:
        """Insert the canonical q-grams of a 2-bit packed sequence (int64/uint64
        GPU tensor of words) cut into n_segments segments of seg_len bases."""
        seq = _device_u64(seq, "seq")
        _check(lib().bbfc_insert_kmers(self.handle, seq.data_ptr(), n_segments, seg_len, q, _stream_handle(stream)))

    def query_kmers(self, seq, n_segments: int, seg_len: int, q: int = 31, out=None, stream=None):
        import torch

        seq = _device_u64(seq, "seq")
        n = kmer_count(n_segments, seg_len, q)
        if out is None:
            out = torch.empty(max(1, (n + 63) // 64), dtype=torch.int64, device=seq.device)
        _check(lib().bbfc_query_kmers(self.handle, seq.data_ptr(), n_segments, seg_len, q, out.data_ptr(),
                                      _stream_handle(stream)))
        return out

    def clear(self, stream=None) -> None:
        _check(lib().bbfc_clear(self.handle, _stream_handle(stream)))

    def bulk_workspace_bytes(self, n: int) -> int:
        b = ctypes.c_uint64()
        _check(lib().bbfc_bulk_insert_workspace(self.handle, n, ctypes.byref(b)))
        return int(b.value)

    def bulk_insert(self, keys, workspace=None, stream=None) -> None:
        """Sequential-semantics insert through the sub-array partition; the
        workspace (a uint8 GPU tensor) is allocated if not given."""
        import torch

        keys = _device_u64(keys, "keys")
        need = self.bulk_workspace_bytes(keys.numel())
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
        _check(lib().bbfc_bulk_insert(self.handle, keys.data_ptr(), keys.numel(), workspace.data_ptr(),
                                      workspace.numel() * workspace.element_size(), _stream_handle(stream)))

    def load_histogram(self, out=None, stream=None):
        """Blocks per popcount j = 0..512 as an int64 GPU tensor of 513."""
        import torch

        if out is None:
            dev = torch.device("cuda", torch.cuda.current_device())
            out = torch.empty(513, dtype=torch.int64, device=dev)
        elif out.numel() < 513:
            raise ValueError("histogram needs 513 entries")
        _check(lib().bbfc_load_histogram(self.handle, out.data_ptr(), _stream_handle(stream)))
        return out[:513]

    def download(self, stream=None):
        """All filter words as a numpy uint64 array (synchronises)."""
        import numpy as np

        out = np.empty(8 * self.n_blocks, dtype=np.uint64)
        _check(lib().bbfc_download(self.handle, out.ctypes.data, _stream_handle(stream)))
        return out

    def upload(self, words, stream=None) -> None:
        import numpy as np

        words = np.ascontiguousarray(words, dtype=np.uint64)
        if words.size != 8 * self.n_blocks:
            raise ValueError("word count must be 8 * n_blocks")
        _check(lib().bbfc_upload(self.handle, words.ctypes.data, _stream_handle(stream)))

    def close(self) -> None:
        if self._h is not None:
            _check(lib().bbfc_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _shape_dict(sh: _Shape) -> dict:
    return {"lanes_per_key": sh.lanes_per_key, "tiles_per_wave": sh.tiles_per_wave,
            "wgs_per_cu": sh.wgs_per_cu, "units_per_grab": sh.units_per_grab, "ms": sh.ms}


class Batch:
    """A plan over several filters, each receiving a fixed number of keys per
    call; keys and answers are concatenated filter after filter (answers of
    each filter start at a 64-bit word)."""

    def __init__(self, filters, n_keys):
        if len(filters) != len(n_keys) or not filters:
            raise ValueError("one key count per filter, at least one filter")
        self._filters = list(filters)  # keep the filters alive
        self.n_keys = [int(v) for v in n_keys]
        hs = (ctypes.c_void_p * len(filters))(*[f.handle.value for f in filters])
        ns = (ctypes.c_uint64 * len(filters))(*self.n_keys)
        h = ctypes.c_void_p()
        _check(lib().bbfc_batch_create(hs, ns, len(filters), ctypes.byref(h)))
        self._h = h
        tk, tw = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().bbfc_batch_layout(h, ctypes.byref(tk), ctypes.byref(tw)))
        self.total_keys, self.total_out_words = tk.value, tw.value
        self.key_offsets, self.out_offsets = [], []
        ko = wo = 0
        for n in self.n_keys:
            self.key_offsets.append(ko)
            self.out_offsets.append(wo)
            ko += n
            wo += (n + 63) // 64

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch is closed")
        return self._h

    def insert(self, keys, stream=None) -> None:
        keys = _device_u64(keys, "keys")
        if keys.numel() < self.total_keys:
            raise ValueError("fewer keys than the plan's layout")
        _check(lib().bbfc_batch_insert(self.handle, keys.data_ptr(), _stream_handle(stream)))

    def query(self, keys, out=None, stream=None):
        import torch

        keys = _device_u64(keys, "keys")
        if keys.numel() < self.total_keys:
            raise ValueError("fewer keys than the plan's layout")
        if out is None:
            out = torch.empty(max(self.total_out_words, 1), dtype=torch.int64, device=keys.device)
        elif out.numel() < self.total_out_words:
            raise ValueError("output too small")
        _check(lib().bbfc_batch_query(self.handle, keys.data_ptr(), out.data_ptr(), _stream_handle(stream)))
        return out

    def set_shape(self, op: int, lanes_per_key: int = 8, tiles_per_wave: int = 1, wgs_per_cu: int = 0,
                  units_per_grab: int | None = None) -> None:
        if units_per_grab is None:  # the plan's defaults
            units_per_grab = 1 if op == OP_INSERT else 8
        _check(lib().bbfc_batch_set_shape(self.handle, op, _Shape(lanes_per_key, tiles_per_wave, wgs_per_cu,
                                                                  units_per_grab, 0.0)))

    def get_shape(self, op: int) -> dict:
        sh = _Shape()
        _check(lib().bbfc_batch_get_shape(self.handle, op, ctypes.byref(sh)))
        return _shape_dict(sh)

    def tune(self, op: int, keys, out=None, reps: int = 3, stream=None) -> dict:
        keys = _device_u64(keys, "keys")
        optr = out.data_ptr() if out is not None else None
        sh = _Shape()
        _check(lib().bbfc_batch_tune(self.handle, op, keys.data_ptr(), optr, reps, _stream_handle(stream),
                                     ctypes.byref(sh)))
        return _shape_dict(sh)

    def close(self) -> None:
        if self._h is not None:
            _check(lib().bbfc_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured batch insert and/or batch query, replayed with launch()."""

    def __init__(self, insert_batch=None, insert_keys=None, query_batch=None, query_keys=None, out=None):
        self._keep = (insert_batch, insert_keys, query_batch, query_keys, out)
        h = ctypes.c_void_p()
        _check(lib().bbfc_graph_create(
            insert_batch.handle if insert_batch is not None else None,
            insert_keys.data_ptr() if insert_keys is not None else None,
            query_batch.handle if query_batch is not None else None,
            query_keys.data_ptr() if query_keys is not None else None,
            out.data_ptr() if out is not None else None, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        if self._h is None:
            raise ValueError("graph is closed")
        _check(lib().bbfc_graph_launch(self._h, _stream_handle(stream)))

    def close(self) -> None:
        if self._h is not None:
            _check(lib().bbfc_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching query server over one resident filter; requests
    are numpy uint64 key arrays in host memory (submit, replay) or 64-bit
    GPU tensors (submit_device, replay_device)."""

    def __init__(self, filt: Filter, n_slots: int | None = None, max_batch_keys: int | None = None,
                 max_pending_keys: int | None = None, poll_us: int | None = None,
                 batch_window_us: int | None = None):
        """Arguments left None take the library's defaults."""
        self._filter = filt
        cfg = _ServerConfig()
        _check(lib().bbfc_server_default_config(ctypes.byref(cfg)))
        for name, v in (("n_slots", n_slots), ("max_batch_keys", max_batch_keys),
                        ("max_pending_keys", max_pending_keys), ("poll_us", poll_us),
                        ("batch_window_us", batch_window_us)):
            if v is not None:
                setattr(cfg, name, int(v))
        self._cfg = {name: int(getattr(cfg, name)) for name, _ in _ServerConfig._fields_}
        h = ctypes.c_void_p()
        _check(lib().bbfc_server_create(filt.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._live = {}  # ticket -> (keys, out) kept alive until waited for

    def config(self) -> dict:
        """The configuration the server was created with."""
        return dict(self._cfg)

    def submit(self, keys) -> int:
        import numpy as np

        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(max(1, (len(keys) + 63) // 64), dtype=np.uint64)
        t = ctypes.c_uint64()
        _check(lib().bbfc_server_submit(self._h, keys.ctypes.data, len(keys), out.ctypes.data, ctypes.byref(t)))
        self._live[t.value] = (keys, out)
        return t.value

    def submit_device(self, keys, out=None) -> int:
        """Submit a request whose keys are a GPU tensor; its packed answers
        are written to `out` (an int64 GPU tensor of ceil(n/64) words,
        allocated if not given) by the server's query launch."""
        import torch

        keys = _device_u64(keys, "keys")
        n = keys.numel()
        if out is None:
            out = torch.zeros(max(1, (n + 63) // 64), dtype=torch.int64, device=keys.device)
        out = _device_u64(out, "out")
        if out.numel() < (n + 63) // 64:
            raise ValueError("output too small")
        t = ctypes.c_uint64()
        _check(lib().bbfc_server_submit_device(self._h, keys.data_ptr(), n, out.data_ptr(), ctypes.byref(t)))
        self._live[t.value] = (keys, out)
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0):
        """(packed answer words, latency in microseconds); the words are a
        numpy array for host requests and a GPU tensor for device ones."""
        lat = ctypes.c_double()
        _check(lib().bbfc_server_wait(self._h, ticket, timeout_s, ctypes.byref(lat)))
        keys, out = self._live.pop(ticket)
        n = keys.numel() if hasattr(keys, "numel") else len(keys)
        return out[: (n + 63) // 64], lat.value

    def replay_device(self, keys, req_offsets, arrival_s, out=None):
        """replay with the keys in a GPU tensor: request i reads
        keys[req_offsets[i]:req_offsets[i+1]] in place and its answers go to
        a GPU tensor (word offsets as in replay). Returns (answer tensor,
        word offsets, latencies in us, wall s)."""
        import numpy as np
        import torch

        keys = _device_u64(keys, "keys")
        ro = np.ascontiguousarray(req_offsets, dtype=np.uint64)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        nreq = len(ro) - 1
        words = (np.diff(ro) + 63) // 64
        oo = np.zeros(nreq + 1, dtype=np.uint64)
        oo[1:] = np.cumsum(words)
        if out is None:
            out = torch.zeros(max(1, int(oo[-1])), dtype=torch.int64, device=keys.device)
        out = _device_u64(out, "out")
        if out.numel() < int(oo[-1]):
            raise ValueError("output too small")
        lat = np.zeros(nreq, dtype=np.float64)
        wall = ctypes.c_double()
        _check(lib().bbfc_server_replay_device(self._h, keys.data_ptr(), ro.ctypes.data, nreq, arr.ctypes.data,
                                               out.data_ptr(), oo.ctypes.data, lat.ctypes.data, ctypes.byref(wall)))
        return out, oo, lat, wall.value

    def stats(self) -> dict:
        b, k, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().bbfc_server_stats(self._h, ctypes.byref(b), ctypes.byref(k), ctypes.byref(c)))
        return {"batches": b.value, "batched_keys": k.value, "completed": c.value}

    def replay(self, keys, req_offsets, arrival_s):
        """Submit request i (keys[req_offsets[i]:req_offsets[i+1]]) at
        arrival_s[i]; returns (answers per request, latencies in us, wall s)."""
        import numpy as np

        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        ro = np.ascontiguousarray(req_offsets, dtype=np.uint64)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        nreq = len(ro) - 1
        words = (np.diff(ro) + 63) // 64
        oo = np.zeros(nreq + 1, dtype=np.uint64)
        oo[1:] = np.cumsum(words)
        out = np.zeros(max(1, int(oo[-1])), dtype=np.uint64)
        lat = np.zeros(nreq, dtype=np.float64)
        wall = ctypes.c_double()
        _check(lib().bbfc_server_replay(self._h, keys.ctypes.data, ro.ctypes.data, nreq, arr.ctypes.data,
                                        out.ctypes.data, oo.ctypes.data, lat.ctypes.data, ctypes.byref(wall)))
        answers = [out[int(oo[i]):int(oo[i + 1])] for i in range(nreq)]
        return answers, lat, wall.value

    def close(self) -> None:
        if self._h is not None:
            _check(lib().bbfc_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- measurement hooks

def probe_gather(buf, n_access: int, seed: int, sink, access_bytes: int = 64, stream=None) -> None:
    if sink.numel() < 65536:
        raise ValueError("probe sink needs at least 65536 words")
    n_lines = buf.numel() // 8
    if n_lines & (n_lines - 1) or n_lines < 2:
        raise ValueError("probe buffer must hold a power-of-two number (>= 2) of 64-byte lines")
    _check(lib().bbfc_probe_gather(buf.data_ptr(), n_lines, access_bytes, n_access, seed, sink.data_ptr(),
                                   _stream_handle(stream)))


def probe_atomic64(buf, n_access: int, seed: int, stream=None) -> None:
    n_lines = buf.numel() // 8
    if n_lines & (n_lines - 1):
        raise ValueError("probe buffer must hold a power-of-two number of 64-byte lines")
    _check(lib().bbfc_probe_atomic64(buf.data_ptr(), n_lines, n_access, seed, _stream_handle(stream)))


def probe_insert_pattern(buf, n_keys: int, mask_bits: int, seed: int, sink, stream=None) -> None:
    """Two random line reads per key, and with ``mask_bits`` > 0 a dependent
    atomic OR of a ``mask_bits``-bit mask into one of the lines (see bbfc.h)."""
    n_lines = buf.numel() // 8
    _check(lib().bbfc_probe_insert_pattern(buf.data_ptr(), n_lines, n_keys, int(mask_bits), seed, sink.data_ptr(),
                                           _stream_handle(stream)))


def probe_insert_schedule(buf, n_keys: int, mask_bits: int, schedule: int, seed: int, sink, stream=None) -> None:
    """The insert's pattern under schedule 0 (reads, then atomics), 1
    (pipelined) or 2 (line chosen without the reads; see bbfc.h)."""
    n_lines = buf.numel() // 8
    _check(lib().bbfc_probe_insert_schedule(buf.data_ptr(), n_lines, n_keys, int(mask_bits), int(schedule), seed,
                                            sink.data_ptr(), _stream_handle(stream)))


def probe_latency(buf, kind: int, out, iters: int = 2000, stream=None) -> None:
    """Mean nanoseconds per dependent step of one memory round trip, one
    wavefront per entry of out (a float64 device tensor): kind 0 line read,
    1 atomic OR, 2 read then atomic OR on that line, 3 key-stream load (see
    bbfc.h)."""
    if out.dtype.itemsize != 8 or not out.is_contiguous():
        raise BBFCError(-1, "out must be a contiguous float64 tensor")
    n_lines = buf.numel() // 8
    _check(lib().bbfc_probe_latency(buf.data_ptr(), n_lines, int(kind), int(iters), out.numel(), out.data_ptr(),
                                    _stream_handle(stream)))


def probe_copy(src, dst, request_bytes: int = 128, stream=None) -> None:
    n = min(src.numel(), dst.numel())
    _check(lib().bbfc_probe_copy(src.data_ptr(), dst.data_ptr(), n, request_bytes, _stream_handle(stream)))


def unpack_bits(words, n: int):
    """Packed answer words (torch or numpy) to a numpy bool array of length n."""
    import numpy as np

    if hasattr(words, "cpu"):
        words = words.cpu().numpy()
    w = np.ascontiguousarray(words).view(np.uint64)
    return np.unpackbits(w.view(np.uint8), bitorder="little")[:n].astype(bool)

