// Shared host/device definitions of the filter library (not part of the ABI).
//
// Hashing follows Section 3.4 of the paper: x -> ((a*x) mod 2^64) mod b, where
// for b = 2^s the s most significant bits of a*x are used, and for even b
// that is not a power of two the high 32 bits are xor-folded into the low
// bits before the remainder. Keys are always treated as 64-bit words.
#pragma once

#include <stdint.h>

#include <utility>

#include <hip/hip_runtime.h>

#include "../../include/bbfc.h"

namespace bbfc {

// How the linear hash reduces a*x into [0, b).
enum HashMode : int {
    kModeOne = 0,  // b == 1: every key maps to 0
    kModePow2 = 1, // b == 2^s: top s bits
    kModeEven = 2, // b even, not 2^s: fold, then remainder
    kModeOdd = 3,  // b odd: remainder
};

// Remainder by an invariant 64-bit divisor d >= 1 without a division
// instruction: Granlund and Montgomery, "Division by invariant integers
// using multiplication" (PLDI 1994), Fig. 4.1 with N = 64:
//   l = ceil(log2 d), m' = floor(2^64 (2^l - d) / d) + 1,
//   t = mulhi(m', n), q = (t + ((n - t) >> sh1)) >> sh2,
//   sh1 = min(l, 1), sh2 = max(l - 1, 0);  r = n - q d.
struct FastMod {
    uint64_t d;
    uint64_t magic;
    uint32_t sh1;
    uint32_t sh2;
};

inline FastMod make_fastmod(uint64_t d)
{
    FastMod fm{};
    fm.d = d;
    uint32_t l = 0;
    while (l < 64 && (((unsigned __int128)1 << l) < d))
        l++;
    unsigned __int128 two_l = (unsigned __int128)1 << l;
    unsigned __int128 num = (((unsigned __int128)1) << 64) * (two_l - d);
    fm.magic = (uint64_t)(num / d + 1);
    fm.sh1 = l < 1 ? l : 1;
    fm.sh2 = l > 0 ? l - 1 : 0;
    return fm;
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ __forceinline__ uint64_t fastdiv(uint64_t n, uint64_t magic, uint32_t sh1, uint32_t sh2)
{
    const uint64_t t = mulhi64(magic, n);
    return (t + ((n - t) >> sh1)) >> sh2;
}

__host__ __device__ __forceinline__ uint64_t fastmod(uint64_t n, uint64_t d, uint64_t magic, uint32_t sh1, uint32_t sh2)
{
    uint64_t t = mulhi64(magic, n);
    uint64_t q = (t + ((n - t) >> sh1)) >> sh2;
    return n - q * d;
}

// A modulus b of the linear hash with what its reduction needs.
struct HashMod {
    uint64_t b;
    uint64_t magic;         // FastMod of b (modes Even, Odd)
    uint32_t sh1;
    uint32_t sh2;
    uint32_t pow2_shift;    // 64 - log2(b) (mode Pow2)
    uint32_t mode;          // HashMode of b
};

inline HashMod make_hashmod(uint64_t b)
{
    HashMod h{};
    h.b = b;
    const FastMod fm = make_fastmod(b);
    h.magic = fm.magic;
    h.sh1 = fm.sh1;
    h.sh2 = fm.sh2;
    if (b == 1) {
        h.mode = kModeOne;
    } else if ((b & (b - 1)) == 0) {
        h.mode = kModePow2;
        h.pow2_shift = 64u - (uint32_t)__builtin_ctzll(b);
    } else {
        h.mode = (b & 1) ? kModeOdd : kModeEven;
    }
    return h;
}

template <int MODE>
__host__ __device__ __forceinline__ uint64_t hash_mod(const HashMod &h, uint64_t a, uint64_t x)
{
    const uint64_t prod = a * x;
    if constexpr (MODE == kModeOne) {
        return 0;
    } else if constexpr (MODE == kModePow2) {
        return prod >> h.pow2_shift;
    } else if constexpr (MODE == kModeEven) {
        return fastmod(prod ^ (prod >> 32), h.b, h.magic, h.sh1, h.sh2);
    } else {
        return fastmod(prod, h.b, h.magic, h.sh1, h.sh2);
    }
}

// The mode read at run time (uniform across a wavefront).
__host__ __device__ __forceinline__ uint64_t hash_mod_rt(const HashMod &h, uint64_t a, uint64_t x)
{
    switch (h.mode) {
    case kModeOne:
        return hash_mod<kModeOne>(h, a, x);
    case kModePow2:
        return hash_mod<kModePow2>(h, a, x);
    case kModeEven:
        return hash_mod<kModeEven>(h, a, x);
    default:
        return hash_mod<kModeOdd>(h, a, x);
    }
}

// Everything a kernel needs to address the filter, passed by value. The M
// blocks form T sub-arrays of S = M/T blocks (Section 3.4, Parallelization):
// h_0(x) (modulus T, multiplier sub_mult) picks the sub-array and the block
// hashes (modulus S) the block inside it. T = 1 is a single array, S = M.
struct KParams {
    uint64_t *words;        // 8*M words, block b = words[8b .. 8b+8)
    const uint16_t *rank;   // (k+1)*513 cost ranks, index a*513 + j
    HashMod blk;            // modulus S of the block hashes h_1..h_c
    HashMod sub;            // modulus T of the sub-array hash h_0
    uint64_t sub_mult;
    uint32_t k;
    uint32_t c;             // choices (informational; kernels take C as a template)
    uint32_t distinct;      // bit selection: 0 random, 1 distinct
    uint64_t block_mult[BBFC_MAX_CHOICES];
    uint64_t bit_mult[BBFC_MAX_BITS_PER_KEY];
};

// Block index inside the key's sub-array, for block multiplier a.
__host__ __device__ __forceinline__ uint64_t block_hash_rt(const KParams &p, uint64_t a, uint64_t x)
{
    return hash_mod_rt(p.blk, a, x);
}

// First block of the key's sub-array: h_0(x) * S (0 for a single array).
__host__ __device__ __forceinline__ uint64_t sub_base(const KParams &p, uint64_t x)
{
    return p.sub.b == 1 ? 0 : hash_mod_rt(p.sub, p.sub_mult, x) * p.blk.b;
}

// Bit address in [0, 512): the top 9 bits of a*x (b = 512 = 2^9).
__host__ __device__ __forceinline__ uint32_t bit_hash(uint64_t a, uint64_t x)
{
    return (uint32_t)((a * x) >> 55);
}

// ------------------------------------------------- distinct bit selection
//
// Section 3.3 / App. B: the i-th value (i counted from 0) is hashed into
// [512 - i] and then names the raw-th address not taken by the earlier ones,
// so a key gets exactly k distinct addresses, a uniform k-subset of [512].
// The paper reaches that address by insertion sort. Here each earlier
// address s keeps fb(s), the number of free addresses below it; s lies
// below the new address v exactly when fb(s) <= raw, so
//     v = raw + #{ s : fb(s) <= raw },
// and afterwards every s above v loses one free address below it. That is
// k(k-1)/2 independent compare/add pairs with no data-dependent indexing.

// Granlund-Montgomery magic for a divisor d in (256, 512] (l = 9):
// floor(2^64 (512 - d) / d) + 1 by binary long division.
constexpr uint64_t small_magic(uint64_t d)
{
    uint64_t q = 0;
    uint64_t rem = 512 - d;
    for (int b = 0; b < 64; ++b) {
        rem <<= 1;
        q <<= 1;
        if (rem >= d) {
            rem -= d;
            q |= 1;
        }
    }
    return q + 1;
}

// f_i(x) into [512 - I] with the hash of Section 3.4 (I = 0: top 9 bits).
template <uint32_t I>
__host__ __device__ __forceinline__ uint32_t distinct_raw(uint64_t a, uint64_t x)
{
    const uint64_t prod = a * x;
    if constexpr (I == 0) {
        return (uint32_t)(prod >> 55);
    } else {
        constexpr uint64_t d = 512 - I;
        constexpr uint64_t magic = small_magic(d);
        const uint64_t n = (d & 1) ? prod : (prod ^ (prod >> 32));
        return (uint32_t)fastmod(n, d, magic, 1, 8);
    }
}

template <uint32_t I, typename Emit>
__host__ __device__ __forceinline__ void distinct_step(uint64_t a, uint64_t x, uint32_t (&fb)[BBFC_MAX_BITS_PER_KEY],
                                              Emit &emit)
{
    const uint32_t raw = distinct_raw<I>(a, x);
    uint32_t v = raw;
#pragma unroll
    for (uint32_t j = 0; j < I; ++j) {
        const bool below = fb[j] <= raw;
        v += below ? 1u : 0u;
        fb[j] -= below ? 0u : 1u;
    }
    fb[I] = raw;
    emit(v);
}

template <typename Emit, uint32_t... I>
__host__ __device__ __forceinline__ void distinct_bits_seq(const uint64_t *mult, uint32_t k, uint64_t x, Emit &emit,
                                                  std::integer_sequence<uint32_t, I...>)
{
    uint32_t fb[BBFC_MAX_BITS_PER_KEY];
    (void)((I < k ? (distinct_step<I>(mult[I], x, fb, emit), true) : false) && ...);
}

// Calls emit(v) once for each of the k distinct addresses of key x.
template <typename Emit>
__host__ __device__ __forceinline__ void distinct_bits(const uint64_t *mult, uint32_t k, uint64_t x, Emit &&emit)
{
    distinct_bits_seq(mult, k, x, emit, std::make_integer_sequence<uint32_t, BBFC_MAX_BITS_PER_KEY>{});
}

// Calls emit(f_i(x)) for the k random-strategy addresses (may repeat).
template <typename Emit>
__host__ __device__ __forceinline__ void random_bits(const uint64_t *mult, uint32_t k, uint64_t x, Emit &&emit)
{
#pragma unroll
    for (int i = 0; i < (int)BBFC_MAX_BITS_PER_KEY; ++i)
        if ((uint32_t)i < k)
            emit(bit_hash(mult[i], x));
}

} // namespace bbfc
