// Device building blocks of the insert and query kernels, shared by the
// single-filter kernels and the batched persistent kernels.
//
// A wavefront works on tiles of 64 keys.
//
//   Phase A, one lane per key. Lane t loads key t of the tile (a coalesced
//   512-byte read), computes the k bit addresses f_i(x) (Section 3.3,
//   random strategy) and ORs each bit into the key's 512-bit mask slot in
//   LDS with ds_or_b32, and computes the c block indices h_i(x)
//   (Section 3.4), stored beside the masks. The bit addresses are computed
//   once per key and reused for every choice, as Section 3.4 recommends.
//
//   Phase B, LPK lanes per key (LPK = 8 or 4). Lane (g, l) = (lane / LPK,
//   lane % LPK) works on tile key g*LPK + r in round r = 0..LPK-1 and owns
//   the 8/LPK consecutive 64-bit words starting at word (8/LPK)*l of each of
//   the key's candidate blocks and of its mask, so the LPK lanes of a group
//   together read one aligned 64-byte block with one request. Every block
//   load of the T tiles a wavefront holds is issued before any is used (the
//   GPU form of prefetching every choice, Section 3.4).
//
//   Query: a block holds F(x) iff (B & m) == m in all lanes of the group;
//   the AND over the group and the OR over choices are taken on the
//   wavefront ballot, and bit t of the tile's answer word answers tile key
//   t (key g*LPK + r lands on bit g*LPK + r, so a shift by r places a round).
//
//   Insert: per candidate, popcount(B | m) and popcount(m & ~B) give each
//   lane's share of j and a (Section 3.2); DPP sums over the group give j and
//   a of every candidate at once. A candidate with a == 0 already holds
//   F(x): no write. Otherwise the candidate of smallest cost rank (ties: the
//   lowest index) receives the mask, one 64-bit atomic OR per word that
//   gains bits.
//
// Costs are never evaluated on the device: the host turns the double-valued
// cost into a dense integer rank table over (j, a), so comparing ranks is
// comparing the doubles exactly.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "bbfc_common.hpp"

namespace bbfc {

constexpr int kWave = 64;
constexpr int kTile = 64;        // keys per tile, one per lane in phase A
constexpr int kSlotDw = 18;      // LDS dwords per key mask (16 used; stride 18 spreads a
                                 // round's groups over disjoint bank pairs)
constexpr int kRankStride = 513; // j in [0, 512]

__device__ __forceinline__ void wave_sync()
{
    // LDS operations of one wavefront execute in order; this only keeps the
    // compiler from moving LDS accesses across the phase boundary.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over each aligned group of LPK (4 or 8) lanes, result in every lane.
template <int LPK>
__device__ __forceinline__ uint32_t group_sum(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false); // quad_perm 1,0,3,2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false); // quad_perm 2,3,0,1
    if constexpr (LPK == 8)
        v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false); // row_half_mirror
    return v;
}

// Bit LPK*g of the result is the AND of the LPK ballot bits of group g.
template <int LPK>
__device__ __forceinline__ uint64_t group_all(uint64_t b)
{
    b &= b >> 1;
    b &= b >> 2;
    if constexpr (LPK == 8)
        b &= b >> 4;
    return b;
}

template <int LPK>
struct Lanes {
    static_assert(LPK == 4 || LPK == 8, "lanes per key must be 4 or 8");
    static constexpr int kGroups = kWave / LPK;     // keys per round
    static constexpr int kRounds = kTile / kGroups; // rounds per tile (== LPK)
    static constexpr int kWords = 8 / LPK;          // 64-bit words a lane owns per block
    static constexpr uint64_t kLsb = LPK == 8 ? 0x0101010101010101ull : 0x1111111111111111ull;
};

__device__ __forceinline__ uint32_t popc64(uint64_t v)
{
    return (uint32_t)__popcll(v);
}

// Key sources: key t of a call, read from an array or computed in place.
struct ArrayKeys {
    const uint64_t *__restrict__ keys;
    __device__ inline uint64_t load(uint64_t t) const { return keys[t]; }
    __device__ inline ArrayKeys offset(uint64_t off) const { return ArrayKeys{keys + off}; }
};

// Canonical q-grams (k-mers of q bases) of a 2-bit packed sequence (A=0, C=1, G=2, T=3; base i in
// bits 63-2(i%32) .. 62-2(i%32) of word i/32, so earlier bases sit higher)
// cut into segments of seg_len bases: key t is the window at base
// s*seg_len + j with s = t / per_seg, j = t % per_seg, per_seg = seg_len-q+1.
// A window's forward value has its first base most significant; the reverse
// complement complements each base (b -> 3-b) and reverses their order; the
// key is the smaller of the two.
struct KmerKeys {
    const uint64_t *__restrict__ seq;
    uint64_t seg_len;
    uint64_t per_seg;
    uint64_t fm_magic; // FastMod of per_seg
    uint32_t fm_sh1;
    uint32_t fm_sh2;
    uint32_t q; // bases per window (1..32)
    __device__ inline uint64_t load(uint64_t t) const
    {
        const uint64_t s = per_seg == 1 ? t : fastdiv(t, fm_magic, fm_sh1, fm_sh2);
        const uint64_t pos = s * seg_len + (t - s * per_seg);
        const uint64_t w = pos >> 5;
        const uint32_t o = (uint32_t)(pos & 31);
        uint64_t v = seq[w];
        if (o != 0) {
            v <<= 2 * o;
            if (o + q > 32) // the window reaches into the next word
                v |= seq[w + 1] >> (64 - 2 * o);
        }
        const uint64_t fwd = v >> (64 - 2 * q);
        // bit reversal reverses the bases and the two bits of each base;
        // swapping the bits of every pair back leaves the bases reversed
        uint64_t r = __builtin_bitreverse64(~fwd);
        r = ((r >> 1) & 0x5555555555555555ull) | ((r & 0x5555555555555555ull) << 1);
        const uint64_t rc = r >> (64 - 2 * q);
        return fwd < rc ? fwd : rc;
    }
};

// Phase A: lane t handles key base + t; keys past n are hashed as key 0,
// whose candidate blocks are in range, so later loads need no guard.
template <int C, typename Src>
__device__ __forceinline__ void phase_a(const KParams &p, const Src &src, uint64_t n, uint64_t base, uint32_t lane,
                               uint32_t *smask, uint64_t *sblk)
{
    const uint64_t idx = base + lane;
    uint64_t x = 0;
    if (idx < n)
        x = src.load(idx);
    uint32_t *slot = smask + lane * kSlotDw;
#pragma unroll
    for (int d = 0; d < 16; ++d)
        slot[d] = 0;
    auto set_bit = [slot](uint32_t f) { atomicOr(slot + (f >> 5), 1u << (f & 31)); };
    if (p.distinct)
        distinct_bits(p.bit_mult, p.k, x, set_bit);
    else
        random_bits(p.bit_mult, p.k, x, set_bit);
    const uint64_t first = sub_base(p, x);
#pragma unroll
    for (int i = 0; i < C; ++i)
        sblk[lane * C + i] = first + block_hash_rt(p, p.block_mult[i], x);
}

template <int KW>
__device__ __forceinline__ void mask_words(const uint32_t *smask, uint32_t t, uint32_t w0, uint64_t (&m)[KW])
{
#pragma unroll
    for (int q = 0; q < KW; ++q) {
        const uint32_t *s = smask + t * kSlotDw + 2 * (w0 + q);
        m[q] = (uint64_t)s[0] | ((uint64_t)s[1] << 32);
    }
}

// Words w0 .. w0+KW-1 of a block (16-byte aligned when KW == 2).
template <int KW>
__device__ __forceinline__ void load_block(const uint64_t *src, uint64_t (&B)[KW])
{
    if constexpr (KW == 1) {
        B[0] = src[0];
    } else {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(src);
        B[0] = v.x;
        B[1] = v.y;
    }
}

template <int KW>
__device__ __forceinline__ bool holds(const uint64_t (&B)[KW], const uint64_t (&m)[KW])
{
    bool ok = true;
#pragma unroll
    for (int q = 0; q < KW; ++q)
        ok &= (B[q] & m[q]) == m[q];
    return ok;
}

// ------------------------------------------------------------------ query

// Answers for T consecutive tiles whose first key is keys[base]; keys past n
// answer false. out_tile[tt] receives the packed answers of tile tt for each
// tile that holds at least one key. EARLY: candidate i+1 is read only by the
// groups whose key candidates 1..i did not answer (same answers, fewer
// random lines).
template <int C, int LPK, int T, bool EARLY, typename Src>
__device__ __forceinline__ void query_tiles(const KParams &p, const Src &keys, uint64_t n, uint64_t base,
                                   uint64_t *__restrict__ out_tile, uint32_t lane, uint32_t *smask, uint64_t *sblk)
{
    using L = Lanes<LPK>;
    constexpr int R = L::kRounds;
    constexpr int KW = L::kWords;
    const uint32_t g = lane / LPK;
    const uint32_t w0 = (lane % LPK) * KW;

    for (int tt = 0; tt < T; ++tt) // T = 1 or 2; phase A writes only LDS, no registers carry over
        phase_a<C>(p, keys, n, base + (uint64_t)tt * kTile, lane, smask + tt * kTile * kSlotDw, sblk + tt * kTile * C);
    wave_sync();

    uint64_t m[T][R][KW];
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
#pragma unroll
        for (int r = 0; r < R; ++r)
            mask_words<KW>(smask + tt * kTile * kSlotDw, g * R + r, w0, m[tt][r]);

    // Bit g*R + r of found[tt]: tile key g*R + r is in a block tested so far.
    uint64_t found[T];
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
        found[tt] = 0;

    if constexpr (!EARLY || C == 1) {
        uint64_t B[T][R][C][KW];
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int i = 0; i < C; ++i)
                    load_block<KW>(p.words + sblk[tt * kTile * C + (g * R + r) * C + i] * 8 + w0, B[tt][r][i]);
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                uint64_t hit = 0;
#pragma unroll
                for (int i = 0; i < C; ++i)
                    hit |= group_all<LPK>(__ballot(holds<KW>(B[tt][r][i], m[tt][r])));
                found[tt] |= (hit & L::kLsb) << r;
            }
    } else {
        uint64_t B[T][R][KW];
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int r = 0; r < R; ++r)
                load_block<KW>(p.words + sblk[tt * kTile * C + (g * R + r) * C] * 8 + w0, B[tt][r]);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            if (i > 0) {
#pragma unroll
                for (int tt = 0; tt < T; ++tt)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (!((found[tt] >> (g * R + r)) & 1))
                            load_block<KW>(p.words + sblk[tt * kTile * C + (g * R + r) * C + i] * 8 + w0, B[tt][r]);
            }
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    found[tt] |= (group_all<LPK>(__ballot(holds<KW>(B[tt][r], m[tt][r]))) & L::kLsb) << r;
        }
    }
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const uint64_t tb = base + (uint64_t)tt * kTile;
        if (tb < n) {
            const uint64_t rem = n - tb;
            uint64_t word = found[tt];
            if (rem < 64)
                word &= (1ull << rem) - 1;
            if (lane == 0)
                out_tile[tt] = word;
        }
    }
    wave_sync();
}

// ----------------------------------------------------------------- insert

// j and a of every candidate, summed over the group. Each candidate takes 16
// bits: j in bits 6..15 (<= 512), a in bits 0..5 (<= k <= 32); every partial
// sum is at most the total, so no field carries into the next.
template <int C>
struct JA {
    uint32_t packed[(C + 1) / 2];
    __device__ inline uint32_t j(int i) const { return (packed[i >> 1] >> (16 * (i & 1) + 6)) & 0x3FF; }
    __device__ inline uint32_t a(int i) const { return (packed[i >> 1] >> (16 * (i & 1))) & 0x3F; }
};

template <int C, int LPK, int KW>
__device__ __forceinline__ JA<C> reduce_ja(const uint64_t (&B)[C][KW], const uint64_t (&m)[KW])
{
    JA<C> r;
#pragma unroll
    for (int h = 0; h < (C + 1) / 2; ++h)
        r.packed[h] = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        uint32_t jj = 0, aa = 0;
#pragma unroll
        for (int q = 0; q < KW; ++q) {
            jj += popc64(B[i][q] | m[q]);
            aa += popc64(m[q] & ~B[i][q]);
        }
        r.packed[i >> 1] |= ((jj << 6) | aa) << (16 * (i & 1));
    }
#pragma unroll
    for (int h = 0; h < (C + 1) / 2; ++h)
        r.packed[h] = group_sum<LPK>(r.packed[h]);
    return r;
}

// Choice receiving the key, or -1 if some candidate already holds F(x).
template <int C>
__device__ __forceinline__ int decide(const JA<C> &ja, const uint16_t *rank)
{
    bool present = false;
#pragma unroll
    for (int i = 0; i < C; ++i)
        present |= ja.a(i) == 0;
    if (present)
        return -1;
    if constexpr (C == 1) {
        return 0;
    } else {
        int best = 0;
        uint32_t rb = rank[ja.a(0) * kRankStride + ja.j(0)];
#pragma unroll
        for (int i = 1; i < C; ++i) {
            const uint32_t ri = rank[ja.a(i) * kRankStride + ja.j(i)];
            if (ri < rb) { // strict: the first minimum wins
                best = i;
                rb = ri;
            }
        }
        return best;
    }
}

__device__ __forceinline__ void atomic_or_word(uint64_t *addr, uint64_t v)
{
    __hip_atomic_fetch_or(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// B[i][q] selected with masks rather than an index, so the candidates stay in
// registers (an indexed select would be lowered to a private-memory array).
template <int C, int KW>
__device__ __forceinline__ uint64_t pick(const uint64_t (&B)[C][KW], int i, int q)
{
    uint64_t v = 0;
#pragma unroll
    for (int c = 0; c < C; ++c)
        v |= B[c][q] & (0ull - (uint64_t)(i == c));
    return v;
}

// Racing insert of T consecutive tiles whose first key is keys[base].
// REC: rec[t] also receives key t's decision, the index of the candidate
// that received F(x) or kPresent when a candidate already held it (a
// checking aid; the kernels that are timed do not record).
constexpr uint8_t kPresent = 0xFF;

template <int C, int LPK, int T, typename Src, bool REC = false>
__device__ __forceinline__ void insert_tiles(const KParams &p, const uint16_t *rank, const Src &keys, uint64_t n,
                                    uint64_t base, uint32_t lane, uint32_t *smask, uint64_t *sblk,
                                    uint8_t *__restrict__ rec = nullptr)
{
    using L = Lanes<LPK>;
    constexpr int R = L::kRounds;
    constexpr int KW = L::kWords;
    const uint32_t g = lane / LPK;
    const uint32_t w0 = (lane % LPK) * KW;

    for (int tt = 0; tt < T; ++tt) // T = 1 or 2; phase A writes only LDS, no registers carry over
        phase_a<C>(p, keys, n, base + (uint64_t)tt * kTile, lane, smask + tt * kTile * kSlotDw, sblk + tt * kTile * C);
    wave_sync();

    uint64_t B[T][R][C][KW];
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < C; ++i)
                load_block<KW>(p.words + sblk[tt * kTile * C + (g * R + r) * C + i] * 8 + w0, B[tt][r][i]);
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t t = g * R + r;
            uint64_t m[KW];
            mask_words<KW>(smask + tt * kTile * kSlotDw, t, w0, m);
            const JA<C> ja = reduce_ja<C, LPK, KW>(B[tt][r], m);
            const int best = decide<C>(ja, rank);
            if constexpr (REC) {
                if (w0 == 0 && base + (uint64_t)tt * kTile + t < n)
                    rec[base + (uint64_t)tt * kTile + t] = best < 0 ? kPresent : (uint8_t)best;
            }
            if (best >= 0 && base + (uint64_t)tt * kTile + t < n) {
                const uint64_t blk = sblk[tt * kTile * C + t * C + best];
#pragma unroll
                for (int q = 0; q < KW; ++q)
                    if (m[q] & ~pick<C, KW>(B[tt][r], best, q))
                        atomic_or_word(p.words + blk * 8 + w0 + q, m[q]);
            }
        }
    wave_sync();
}

// Narrow racing insert: a wavefront holds 8 keys, lane (g, l) = (lane / 8,
// lane % 8) works on key g and owns word l of its blocks and mask, and each
// step of a key is spread over its 8 lanes, so one tile is a single round:
// lane l computes the bit addresses f_i with i = l mod 8 (am[j] holds the
// multiplier of f_(8j+l), zero past k) and ORs them into the key's mask slot
// in LDS; each lane computes the key's c block indices itself; the 8 lanes
// read one block together; DPP sums give j and a (Section 3.2). For inserts
// whose keys in flight are few (small filters), where a tile's time is the
// latency of its own instructions and memory round trips rather than
// bandwidth. The distinct strategy (App. B) draws its addresses in order, so
// lane 0 of each group draws them all.
constexpr int kNarrowKeys = 8; // keys per wavefront tile

template <int C, typename Src, bool REC = false>
__device__ __forceinline__ void insert_narrow_tile(const KParams &p, const uint16_t *rank, const Src &keys, uint64_t n,
                                                   uint64_t base, uint32_t lane, const uint64_t (&am)[4],
                                                   uint32_t *smask, uint8_t *__restrict__ rec = nullptr)
{
    const uint32_t g = lane / 8;
    const uint32_t l = lane % 8;
    const uint64_t t = base + g;
    const bool live = t < n;
    const uint64_t x = live ? keys.load(t) : 0; // past n: key 0, whose blocks are in range
    uint32_t *slot = smask + g * kSlotDw;
    slot[2 * l] = 0;
    slot[2 * l + 1] = 0;
    wave_sync();
    auto set_bit = [slot](uint32_t f) { atomicOr(slot + (f >> 5), 1u << (f & 31)); };
    if (p.distinct) {
        if (l == 0)
            distinct_bits(p.bit_mult, p.k, x, set_bit);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (8 * j + l < p.k)
                set_bit(bit_hash(am[j], x));
    }
    const uint64_t first = sub_base(p, x);
    uint64_t blk[C];
#pragma unroll
    for (int i = 0; i < C; ++i)
        blk[i] = first + block_hash_rt(p, p.block_mult[i], x);
    uint64_t B[C][1];
#pragma unroll
    for (int i = 0; i < C; ++i)
        B[i][0] = p.words[blk[i] * 8 + l];
    wave_sync();
    uint64_t m[1];
    m[0] = (uint64_t)slot[2 * l] | ((uint64_t)slot[2 * l + 1] << 32);
    const JA<C> ja = reduce_ja<C, 8, 1>(B, m);
    const int best = decide<C>(ja, rank);
    if constexpr (REC) {
        if (l == 0 && live)
            rec[t] = best < 0 ? kPresent : (uint8_t)best;
    }
    if (best >= 0 && live) {
        uint64_t b = 0;
#pragma unroll
        for (int i = 0; i < C; ++i)
            b |= blk[i] & (0ull - (uint64_t)(best == i));
        if (m[0] & ~pick<C, 1>(B, best, 0))
            atomic_or_word(p.words + b * 8 + l, m[0]);
    }
    wave_sync();
}

} // namespace bbfc
