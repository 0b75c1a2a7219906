"""Independent pure-Python restatement of the filter for tiny inputs.

TEST INFRASTRUCTURE ONLY. It shares nothing with ``bbfc_oracle.c``: blocks
are Python ``set``s of bit addresses F', a key's addresses F(x) are a
``set``, and j, a come from set union and difference exactly as the paper
defines them (Section 3.2: j = |F' u F(x)|, a = |F(x) \\ F'|). Hashing uses
Python's unbounded integers reduced modulo 2^64 (Section 3.4). The result is
converted to 64-bit words only at the end, so the word layout of the C
oracle is checked too.
"""

from __future__ import annotations

import math

U64 = 1 << 64


def lin_hash(a: int, x: int, b: int) -> int:
    """((a*x) mod 2^64) mod b with the even-b modifications of Section 3.4."""
    p = (a * x) % U64
    if b == 1:
        return 0
    s = b.bit_length() - 1
    if (1 << s) == b:
        return p // (1 << (64 - s))  # the s most significant bits of p
    if b % 2 == 0:
        return (p ^ (p // (1 << 32))) % b
    return p % b


def bit_set(bit_mult, x: int) -> set[int]:
    """F(x) = { f_i(x) } with f_i into [512] (eq. bitset, random strategy)."""
    return {lin_hash(a, x, 512) for a in bit_mult}


def bit_set_distinct(bit_mult, x: int) -> set[int]:
    """Distinct strategy (App. B) restated: the i-th raw value, hashed into
    [512 - i], picks that element of the list of addresses still free
    (the paper: a random value from [512] minus the earlier addresses)."""
    free = list(range(512))
    out = set()
    for i, a in enumerate(bit_mult):
        out.add(free.pop(lin_hash(a, x, 512 - i)))
    return out


def cost(kind: str, param: float, k: int, j: int, a: int) -> float:
    """App. A eqs. cost:mix, cost:la, cost:exp (same left-to-right order)."""
    if kind == "mix":
        return param * k * math.pow(j / 256.0, k) + a
    if kind == "la":
        return k * math.pow((j + param * k) / 256.0, k) + a
    if kind == "exp":
        return math.pow(param, j / 128.0) + a / k
    raise ValueError(kind)


class BruteFilter:
    def __init__(self, M: int, c: int, k: int, kind: str, param: float, block_mult, bit_mult,
                 distinct: bool = False, subarrays: int = 1, sub_mult: int = 0):
        self.M, self.c, self.k, self.kind, self.param = M, c, k, kind, param
        self.distinct = distinct
        self.T, self.sub_mult = subarrays, sub_mult  # Section 3.4, Parallelization
        self.block_mult = [int(v) for v in block_mult]
        self.bit_mult = [int(v) for v in bit_mult]
        self.blocks: list[set[int]] = [set() for _ in range(M)]

    def candidates(self, x: int) -> list[int]:
        S = self.M // self.T
        base = S * lin_hash(self.sub_mult, x, self.T)  # sub-array h_0(x), then h_i(x) inside it
        return [base + lin_hash(b, x, S) for b in self.block_mult]

    def F(self, x: int) -> set[int]:
        return bit_set_distinct(self.bit_mult, x) if self.distinct else bit_set(self.bit_mult, x)

    def insert(self, x: int) -> int:
        F = self.F(x)
        cand = self.candidates(x)
        ja = []
        for b in cand:
            Fp = self.blocks[b]
            ja.append((len(Fp | F), len(F - Fp)))
        if any(a == 0 for _, a in ja):
            return -1
        best = 0
        if self.c > 1:
            costs = [cost(self.kind, self.param, self.k, j, a) for j, a in ja]
            best = min(range(self.c), key=lambda i: (costs[i], i))
        self.blocks[cand[best]] |= F
        return best

    def query(self, x: int) -> bool:
        F = self.F(x)
        return any(F <= self.blocks[b] for b in self.candidates(x))

    def words(self) -> list[int]:
        return _words(self.blocks)

    def envelope_words(self, keys) -> list[int]:
        """Every key's F(x) added to every one of its candidates (as sets),
        then converted to words: the largest bit set any schedule of racing
        inserts of these keys could produce (Sections 3.1, 3.2)."""
        env: list[set[int]] = [set() for _ in range(self.M)]
        for x in keys:
            F = self.F(int(x))
            for b in self.candidates(int(x)):
                env[b] |= F
        return _words(env)

    def placed_words(self, keys, decisions) -> list[int]:
        """Blocks as sets after adding each key's F(x) to the one candidate
        its decision names (decision >= c: the key added nothing), Sections
        3.1 and 3.2; converted to words."""
        blocks: list[set[int]] = [set() for _ in range(self.M)]
        for x, d in zip(keys, decisions):
            if int(d) < self.c:
                blocks[self.candidates(int(x))[int(d)]] |= self.F(int(x))
        return _words(blocks)

    def load_counts(self) -> dict[int, int]:
        """Number of blocks per count of set bits |F'| (App. C, load histogram figure)."""
        out: dict[int, int] = {}
        for S in self.blocks:
            out[len(S)] = out.get(len(S), 0) + 1
        return out


def _words(blocks: list[set[int]]) -> list[int]:
    out = []
    for S in blocks:
        for w in range(8):
            out.append(sum(1 << (f - 64 * w) for f in S if f // 64 == w))
    return out
