"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module only draws numbers. It holds none of the filter's arithmetic
(no hashing into blocks or bits, no cost, no popcount): every value it
returns is an input that both the sequential CPU oracle and the HIP library
receive unchanged.

Keys are counter-based SplitMix64 outputs (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014):

    key(seed, i) = mix64(seed + (i + 1) * GAMMA)          (mod 2^64)

``mix64`` is a bijection of 64-bit words and ``GAMMA`` is odd, so for a fixed
seed distinct counters give distinct keys. Positive keys use counters
[0, n) and negative keys [n, 2n): the two sets are disjoint by construction.

Hash multipliers (the "random large integer a, coprime with b" of the
paper's Section 3.4) are drawn here as well for the tests, so that both
sides receive the same parameters as plain inputs.
"""

from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

__all__ = [
    "GAMMA",
    "splitmix64_keys",
    "splitmix64_scalar",
    "SplitMix64",
    "draw_multipliers",
    "positive_keys",
    "negative_keys",
]


def splitmix64_scalar(seed: int, i: int) -> int:
    """key(seed, i) in plain Python integers (used to spot-check samples)."""
    z = (seed + (i + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def splitmix64_keys(seed: int, start: int, n: int) -> np.ndarray:
    """key(seed, start), ..., key(seed, start + n - 1) as a uint64 array.

    numpy's uint64 array arithmetic wraps modulo 2^64, which is exactly the
    generator's definition.
    """
    if n < 0 or start < 0:
        raise ValueError("start and n must be non-negative")
    out = np.empty(n, dtype=np.uint64)
    chunk = 1 << 24
    s = np.uint64(seed & MASK64)
    g = np.uint64(GAMMA)
    m1 = np.uint64(MIX1)
    m2 = np.uint64(MIX2)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        ctr = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
        z = s + ctr * g
        z = (z ^ (z >> np.uint64(30))) * m1
        z = (z ^ (z >> np.uint64(27))) * m2
        out[lo:hi] = z ^ (z >> np.uint64(31))
    return out


def positive_keys(seed: int, n: int) -> np.ndarray:
    """The n keys to insert: counters [0, n)."""
    return splitmix64_keys(seed, 0, n)


def negative_keys(seed: int, n_pos: int, n: int) -> np.ndarray:
    """n keys never inserted: counters [n_pos, n_pos + n)."""
    return splitmix64_keys(seed, n_pos, n)


class SplitMix64:
    """Sequential SplitMix64 stream (state advances by GAMMA per draw)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * MIX1) & MASK64
        z = ((z ^ (z >> 27)) * MIX2) & MASK64
        return z ^ (z >> 31)


def draw_multipliers(seed: int, count: int, coprime_to=2) -> list[int]:
    """``count`` random odd 64-bit multipliers, each >= 2^32 and coprime to
    ``coprime_to`` (one modulus for all, or a sequence with one modulus per
    multiplier); used as hash parameters handed to both sides."""
    mods = [coprime_to] * count if isinstance(coprime_to, int) else [int(m) for m in coprime_to]
    assert len(mods) == count
    rng = SplitMix64(seed ^ 0x5DEECE66D)
    out: list[int] = []
    while len(out) < count:
        a = rng.next() | 1
        if a >= (1 << 32) and math.gcd(a, mods[len(out)]) == 1:
            out.append(a)
    return out


def distinct_moduli(k: int) -> list[int]:
    """Moduli of the k bit hashes under distinct bit selection: 512, 511, ..."""
    return [512 - i for i in range(k)]


def batch_specs(seed: int, count: int, log2_lo: float = 10.0, log2_hi: float = 24.0,
                bits_lo: int = 10, bits_hi: int = 16) -> list[tuple[int, int]]:
    """(keys, space bits per key) of `count` filters: keys = round(2^U) with
    U uniform in [log2_lo, log2_hi], bits uniform in {bits_lo..bits_hi}."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(count):
        u = log2_lo + (log2_hi - log2_lo) * ((rng.next() >> 11) / float(1 << 53))
        b = bits_lo + rng.next() % (bits_hi - bits_lo + 1)
        out.append((int(round(2.0 ** u)), int(b)))
    return out


def serve_requests(seed: int, count: int, n_pos: int, lo: int = 1, hi: int = 65536):
    """A query-request mix: sizes log-uniform in [lo, hi]; each request
    takes half its keys (rounded up) from the n_pos inserted keys (a
    contiguous run of counters at a random start) and the rest from keys
    never inserted (counters from n_pos on, one fresh run per request).
    Returns (sizes, positive starts, negative starts)."""
    rng = SplitMix64(seed)
    sizes, pstart, nstart = [], [], []
    nxt = n_pos
    for _ in range(count):
        u = math.log(lo) + (math.log(hi) - math.log(lo)) * ((rng.next() >> 11) / float(1 << 53))
        s = max(lo, min(hi, int(round(math.exp(u)))))
        npos = (s + 1) // 2
        sizes.append(s)
        pstart.append(rng.next() % max(1, n_pos - npos))
        nstart.append(nxt)
        nxt += s - npos
    return sizes, pstart, nstart


# ------------------------------------------------------------- DNA inputs
# Bases A, C, G, T are the values 0..3. A packed sequence holds 32 bases per
# 64-bit word, base i in bits 63-2(i%32) .. 62-2(i%32) of word i/32.

def genome_packed(seed: int, n_bases: int) -> np.ndarray:
    """A uniform random genome: its packed words are the counter-based
    SplitMix64 outputs key(seed, 0), key(seed, 1), ..."""
    return splitmix64_keys(seed, 0, (n_bases + 31) // 32)


def unpack_2bit(words, n_bases: int) -> np.ndarray:
    """Packed words to one base (0..3) per byte."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    shifts = np.arange(62, -1, -2, dtype=np.uint64)
    b = ((w[:, None] >> shifts[None, :]) & np.uint64(3)).astype(np.uint8).reshape(-1)
    return b[:n_bases]


def pack_2bit(bases) -> np.ndarray:
    """One base (0..3) per byte to packed words (tail bases zero)."""
    b = np.ascontiguousarray(bases, dtype=np.uint64)
    n = len(b)
    pad = np.zeros(((n + 31) // 32) * 32, dtype=np.uint64)
    pad[:n] = b
    shifts = np.arange(62, -1, -2, dtype=np.uint64)
    return np.bitwise_or.reduce(pad.reshape(-1, 32) << shifts[None, :], axis=1)


def random_bases(seed: int, n: int) -> np.ndarray:
    return unpack_2bit(genome_packed(seed, n), n)


_PLANT_ERR_SALT = 0x6B6B6B6B6B6B6B6B
_PLANT_SUB_SALT = 0x1E1E1E1E1E1E1E1E


def repeat_segments(seed: int, n_bases: int, fraction: float, lo: int = 300, hi: int = 6000):
    """Planted repeat segments: lengths log-uniform in [lo, hi], drawn until
    they cover `fraction` of the genome, laid out in draw order with random
    gaps (so they never overlap), each copying from a uniform random source
    position. Returns (dst, length, src) uint64 arrays sorted by dst."""
    rng = SplitMix64(seed ^ 0x7E9E47D3)
    target = int(fraction * n_bases)
    lens = []
    total = 0
    while total < target:
        u = (rng.next() >> 11) / float(1 << 53)
        L = int(round(lo * (hi / lo) ** u))
        L = min(L, n_bases - total)
        if L <= 0:
            break
        lens.append(L)
        total += L
    n = len(lens)
    free = n_bases - total
    cuts = np.sort(np.array([rng.next() % (free + 1) for _ in range(n)], dtype=np.uint64))
    lens_a = np.array(lens, dtype=np.uint64)
    before = np.concatenate([[0], np.cumsum(lens_a)[:-1]]).astype(np.uint64) if n else np.zeros(0, np.uint64)
    dst = cuts + before
    src = np.array([rng.next() % (n_bases - L + 1) for L in lens], dtype=np.uint64)
    return dst, lens_a, src


def plant_numpy(bases, segments, div: float, seed: int) -> np.ndarray:
    """Host restatement of the device planting (one base per byte)."""
    b = np.ascontiguousarray(bases, dtype=np.uint8)
    out = b.copy()
    thr = min(int(div * 2.0 ** 64), MASK64)
    for d, L, s in zip(*segments):
        d, L, s = int(d), int(L), int(s)
        seg = b[s:s + L].astype(np.uint64)
        err = splitmix64_keys(seed ^ _PLANT_ERR_SALT, d, L)
        sub = splitmix64_keys(seed ^ _PLANT_SUB_SALT, d, L)
        flip = err < np.uint64(thr)
        seg = np.where(flip, (seg + np.uint64(1) + sub % np.uint64(3)) & np.uint64(3), seg)
        out[d:d + L] = seg.astype(np.uint8)
    return out


# ----------------------------------------------------- device-side generator

import ctypes as _ctypes
import os as _os
import subprocess as _subprocess

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_DEV_SRC = _os.path.join(_HERE, "csrc", "keygen.hip")
_DEV_LIB = _os.path.join(_HERE, "libworkload.so")
_dev = None


def build_device(arch: str = "gfx950") -> str:
    """Compile the device key generator with hipcc (in-tree)."""
    cmd = ["hipcc", f"--offload-arch={arch}", "-O3", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", _DEV_LIB + ".tmp", _DEV_SRC]
    _subprocess.run(cmd, check=True, stderr=_subprocess.DEVNULL)
    _os.replace(_DEV_LIB + ".tmp", _DEV_LIB)
    return _DEV_LIB


def _device_lib():
    global _dev
    if _dev is None:
        if not _os.path.exists(_DEV_LIB):
            raise RuntimeError(f"{_DEV_LIB} is missing; run workload.build_device()")
        L = _ctypes.CDLL(_DEV_LIB)
        L.wl_splitmix64_keys.argtypes = [_ctypes.c_uint64] * 3 + [_ctypes.c_void_p] * 2
        L.wl_splitmix64_keys.restype = _ctypes.c_int
        L.wl_reads.argtypes = [_ctypes.c_void_p] + [_ctypes.c_uint64] * 5 + [_ctypes.c_void_p] * 2
        L.wl_reads.restype = _ctypes.c_int
        L.wl_plant.argtypes = [_ctypes.c_void_p] * 2 + [_ctypes.c_uint64] + [_ctypes.c_void_p] * 3 + \
            [_ctypes.c_uint64] * 3 + [_ctypes.c_void_p]
        L.wl_plant.restype = _ctypes.c_int
        _dev = L
    return _dev


def device_keys(seed: int, start: int, n: int, device="cuda", out=None, stream=None):
    """key(seed, start .. start+n-1) generated on the GPU into an int64 tensor
    (the same 64-bit patterns as ``splitmix64_keys``)."""
    import torch

    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=device)
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    rc = _device_lib().wl_splitmix64_keys(seed & MASK64, start, n, out.data_ptr(), _ctypes.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"device key generation failed ({rc})")
    return out


def device_reads(genome, n_genome: int, n_reads: int, read_len: int, err: float, seed: int, out=None, stream=None):
    """Packed reads sampled from a packed genome on the GPU (see
    csrc/keygen.hip): uniform start, random strand, substitutions with
    probability err per base."""
    import torch

    n_words = (n_reads * read_len + 31) // 32
    if out is None:
        out = torch.empty(max(1, n_words), dtype=torch.int64, device=genome.device)
    if stream is None:
        stream = torch.cuda.current_stream(genome.device)
    thr = min(int(err * 2.0 ** 64), MASK64)
    rc = _device_lib().wl_reads(genome.data_ptr(), n_genome, n_reads, read_len, thr, seed & MASK64,
                                out.data_ptr(), _ctypes.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"device read generation failed ({rc})")
    return out


def device_plant(genome, n_bases: int, segments, div: float, seed: int, stream=None):
    """A copy of a packed genome on the GPU with the planted repeat segments
    (see repeat_segments / plant_numpy)."""
    import torch

    dst, lens, src = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(genome.device)
                      for a in segments)
    out = torch.empty_like(genome)
    if stream is None:
        stream = torch.cuda.current_stream(genome.device)
    thr = min(int(div * 2.0 ** 64), MASK64)
    rc = _device_lib().wl_plant(genome.data_ptr(), out.data_ptr(), n_bases, dst.data_ptr(), lens.data_ptr(),
                                src.data_ptr(), len(segments[0]), thr, seed & MASK64,
                                _ctypes.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"device repeat planting failed ({rc})")
    stream.synchronize()  # the segment tables are freed on return
    return out
