// Insert and query kernels for Blocked Bloom filters with choices, gfx950.
//
// Work decomposition (one 64-lane wavefront per tile of 64 keys):
//
//   Phase A, one lane per key. Lane t loads key t of the tile (one coalesced
//   512-byte read), computes the k bit addresses f_i(x) (Section 3.3,
//   random strategy) and ORs each bit into the key's 512-bit mask slot in
//   LDS with ds_or_b32, and computes the c block indices h_i(x)
//   (Section 3.4), stored beside the masks. The bit addresses are computed
//   once per key and reused for every choice, as Section 3.4 recommends.
//
//   Phase B, eight lanes per key. Lane (g, w) = (lane/8, lane%8) works on
//   tile key 8g + r in round r = 0..7 and owns 64-bit word w of each of the
//   key's candidate blocks and of its mask. All 8*c block words of the
//   eight rounds are loaded before any is used, so a lane keeps 8c
//   independent loads in flight (the GPU form of prefetching every choice,
//   Section 3.4). Eight lanes reading one 64-byte block issue exactly one
//   aligned 64-byte request.
//
//   Query: a block holds F(x) iff (B_w & m_w) == m_w in all eight lanes;
//   the AND over the lanes and the OR over choices are taken on the
//   wavefront ballot, and bit 8g + r of the tile's output word is the
//   answer for tile key 8g + r, written by lane 0 as one 64-bit store.
//
//   Insert: per candidate, popcount(B_w | m_w) and popcount(B_w) give each
//   lane's share of j and of a = j - |F'| (Section 3.2); a three-step DPP
//   sum over the eight lanes yields j and a for all candidates at once.
//   A candidate with a == 0 already holds F(x): no write. Otherwise the
//   candidate of smallest cost rank (ties: lowest index) receives the mask
//   with one 64-bit atomic OR per word that gains bits.
//
// Costs are never evaluated on the device: the host turns the double-valued
// cost into a dense integer rank table over (j, a), so comparing ranks is
// comparing the doubles exactly.
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "bbfc_common.hpp"
#include "bbfc_internal.hpp"

namespace bbfc {

constexpr int kWave = 64;
constexpr int kTile = 64;            // keys per wavefront tile
constexpr int kSlotDw = 18;          // LDS dwords per key mask (16 used; stride 18 puts
                                     // the eight groups of a round on disjoint bank pairs)
constexpr int kWavesPerWG = 4;
constexpr int kWGSize = kWave * kWavesPerWG;
constexpr int kRankStride = 513;     // j in [0, 512]
constexpr uint64_t kGroupLsb = 0x0101010101010101ull;

__device__ inline void wave_sync()
{
    // LDS operations of one wavefront execute in order; this only keeps the
    // compiler from moving LDS accesses across the phase boundary.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over each aligned group of eight lanes, result in every lane.
__device__ inline uint32_t group8_sum(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false); // row_half_mirror
    return v;
}

__device__ inline uint32_t popc64(uint64_t v)
{
    return (uint32_t)__popcll(v);
}

// Phase A: lane t of the wavefront handles key base + t.
template <int C, int MODE>
__device__ inline void phase_a(const KParams &p, const uint64_t *__restrict__ keys, uint64_t n, uint64_t base,
                               uint32_t lane, uint32_t *smask, uint64_t *sblk)
{
    const uint64_t idx = base + lane;
    uint64_t x = 0;
    if (idx < n)
        x = keys[idx];
    uint32_t *slot = smask + lane * kSlotDw;
#pragma unroll
    for (int d = 0; d < 16; ++d)
        slot[d] = 0;
#pragma unroll
    for (int i = 0; i < (int)BBFC_MAX_BITS_PER_KEY; ++i) {
        if ((uint32_t)i < p.k) {
            const uint32_t f = bit_hash(p.bit_mult[i], x);
            atomicOr(slot + (f >> 5), 1u << (f & 31));
        }
    }
#pragma unroll
    for (int i = 0; i < C; ++i)
        sblk[lane * C + i] = block_hash<MODE>(p, p.block_mult[i], x);
}

__device__ inline uint64_t mask_word(const uint32_t *smask, uint32_t t, uint32_t w)
{
    const uint32_t *q = smask + t * kSlotDw + 2 * w;
    return (uint64_t)q[0] | ((uint64_t)q[1] << 32);
}

// ------------------------------------------------------------------ query

// EARLY: choice i+1 is loaded only by groups whose key none of the choices
// 1..i answered (the answer is the same; fewer random lines are read).
template <int C, int MODE, bool EARLY>
__global__ __launch_bounds__(kWGSize) void query_kernel(KParams p, const uint64_t *__restrict__ keys, uint64_t n,
                                                        uint64_t *__restrict__ out, uint64_t n_tiles)
{
    __shared__ uint32_t s_mask[kWavesPerWG][kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][kTile * C];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    uint32_t *smask = s_mask[wv];
    uint64_t *sblk = s_blk[wv];
    const uint32_t g = lane >> 3;
    const uint32_t w = lane & 7;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerWG;

    for (uint64_t tile = (uint64_t)blockIdx.x * kWavesPerWG + wv; tile < n_tiles; tile += n_waves) {
        const uint64_t base = tile * kTile;
        phase_a<C, MODE>(p, keys, n, base, lane, smask, sblk);
        wave_sync();

        uint64_t m[8];
#pragma unroll
        for (int r = 0; r < 8; ++r)
            m[r] = mask_word(smask, g * 8 + r, w);
        // Bit 8g + r of `found`: tile key 8g + r is in some block tested so far.
        // Keys past n were hashed as key 0, whose blocks are in range, so the
        // loads need no guard; their answers are masked at the end.
        uint64_t found = 0;
        if constexpr (!EARLY || C == 1) {
            uint64_t B[8][C];
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int i = 0; i < C; ++i)
                    B[r][i] = p.words[sblk[(g * 8 + r) * C + i] * 8 + w];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                uint64_t hit = 0;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    uint64_t b = __ballot((B[r][i] & m[r]) == m[r]);
                    b &= b >> 1; // bit 8g: AND of the group's eight lanes after three steps
                    b &= b >> 2;
                    b &= b >> 4;
                    hit |= b;
                }
                found |= (hit & kGroupLsb) << r;
            }
        } else {
            uint64_t B[8];
#pragma unroll
            for (int r = 0; r < 8; ++r)
                B[r] = p.words[sblk[(g * 8 + r) * C] * 8 + w];
#pragma unroll
            for (int i = 0; i < C; ++i) {
                if (i > 0) {
#pragma unroll
                    for (int r = 0; r < 8; ++r)
                        if (!((found >> (g * 8 + r)) & 1))
                            B[r] = p.words[sblk[(g * 8 + r) * C + i] * 8 + w];
                }
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    uint64_t b = __ballot((B[r] & m[r]) == m[r]);
                    b &= b >> 1;
                    b &= b >> 2;
                    b &= b >> 4;
                    found |= (b & kGroupLsb) << r;
                }
            }
        }
        const uint64_t rem = n - base;
        if (rem < 64)
            found &= (1ull << rem) - 1;
        if (lane == 0)
            out[tile] = found;
        wave_sync();
    }
}

// ----------------------------------------------------------------- insert

// j and a of every candidate, reduced over the eight lanes of the group.
// Each candidate takes 16 bits: j in bits 6..15 (<= 512), a in bits 0..5
// (<= k <= 32); per-lane shares are at most 64 and 32, so no field carries.
template <int C>
struct JA {
    uint32_t packed[(C + 1) / 2];
    __device__ inline uint32_t j(int i) const { return (packed[i >> 1] >> (16 * (i & 1) + 6)) & 0x3FF; }
    __device__ inline uint32_t a(int i) const { return (packed[i >> 1] >> (16 * (i & 1))) & 0x3F; }
};

template <int C>
__device__ inline JA<C> reduce_ja(const uint64_t (&B)[C], uint64_t m)
{
    JA<C> r;
#pragma unroll
    for (int h = 0; h < (C + 1) / 2; ++h)
        r.packed[h] = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const uint32_t jj = popc64(B[i] | m);
        const uint32_t aa = jj - popc64(B[i]);
        r.packed[i >> 1] |= ((jj << 6) | aa) << (16 * (i & 1));
    }
#pragma unroll
    for (int h = 0; h < (C + 1) / 2; ++h)
        r.packed[h] = group8_sum(r.packed[h]);
    return r;
}

// Choice receiving the key, or -1 if some candidate already holds F(x).
template <int C>
__device__ inline int decide(const JA<C> &ja, const uint16_t *rank)
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

__device__ inline void atomic_or_word(uint64_t *addr, uint64_t v)
{
    __hip_atomic_fetch_or(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// B[i] selected with masks rather than an index, so the candidates stay in
// registers (an indexed select would be lowered to a private-memory array).
template <int C>
__device__ inline uint64_t pick(const uint64_t (&B)[C], int i)
{
    uint64_t v = 0;
#pragma unroll
    for (int q = 0; q < C; ++q)
        v |= B[q] & (0ull - (uint64_t)(i == q));
    return v;
}

template <int C>
__device__ inline void load_rank_table(const KParams &p, uint16_t *s_rank)
{
    if constexpr (C > 1) {
        const uint32_t n = (p.k + 1) * kRankStride;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
            s_rank[i] = p.rank[i];
    }
    __syncthreads();
}

template <int C, int MODE>
__global__ __launch_bounds__(kWGSize) void insert_kernel(KParams p, const uint64_t *__restrict__ keys, uint64_t n,
                                                         uint64_t n_tiles)
{
    __shared__ uint32_t s_mask[kWavesPerWG][kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][kTile * C];
    extern __shared__ uint16_t s_rank[];
    load_rank_table<C>(p, s_rank);

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    uint32_t *smask = s_mask[wv];
    uint64_t *sblk = s_blk[wv];
    const uint32_t g = lane >> 3;
    const uint32_t w = lane & 7;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerWG;

    for (uint64_t tile = (uint64_t)blockIdx.x * kWavesPerWG + wv; tile < n_tiles; tile += n_waves) {
        const uint64_t base = tile * kTile;
        phase_a<C, MODE>(p, keys, n, base, lane, smask, sblk);
        wave_sync();

        uint64_t B[8][C];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t t = g * 8 + r;
            // Keys past n were hashed as key 0 (blocks in range); they never write.
#pragma unroll
            for (int i = 0; i < C; ++i)
                B[r][i] = p.words[sblk[t * C + i] * 8 + w];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t t = g * 8 + r;
            const uint64_t m = mask_word(smask, t, w);
            const JA<C> ja = reduce_ja<C>(B[r], m);
            const int best = decide<C>(ja, s_rank);
            if (best >= 0 && base + t < n) {
                const uint64_t old = pick<C>(B[r], best);
                if (m & ~old)
                    atomic_or_word(&p.words[sblk[t * C + best] * 8 + w], m);
            }
        }
        wave_sync();
    }
}

// Sequential-semantics insert on a single wavefront. Within a tile the
// keys are taken in index order in windows of up to eight: the window is cut
// before the first key that shares a candidate block with an earlier key of
// the window, so the keys processed together touch disjoint blocks and the
// outcome is that of inserting them one after another. Block words are read
// with agent-scope atomic loads (no stale per-CU cache line) and every
// window's writes complete before the next window reads.
template <int C, int MODE>
__global__ __launch_bounds__(kWave) void insert_det_kernel(KParams p, const uint64_t *__restrict__ keys, uint64_t n,
                                                           uint64_t n_tiles)
{
    __shared__ uint32_t smask[kTile * kSlotDw];
    __shared__ uint64_t sblk[kTile * C];
    extern __shared__ uint16_t s_rank[];
    load_rank_table<C>(p, s_rank);

    const uint32_t lane = threadIdx.x;
    const uint32_t g = lane >> 3;
    const uint32_t w = lane & 7;

    for (uint64_t tile = 0; tile < n_tiles; ++tile) {
        const uint64_t base = tile * kTile;
        phase_a<C, MODE>(p, keys, n, base, lane, smask, sblk);
        wave_sync();
        const uint32_t in_tile = (uint32_t)((n - base) < (uint64_t)kTile ? (n - base) : (uint64_t)kTile);
        uint32_t pos = 0;
        while (pos < in_tile) {
            const uint32_t t = pos + g;
            const bool active = t < in_tile;
            bool conflict = false;
            if (active) {
                for (uint32_t q = 0; q < g; ++q) {
#pragma unroll
                    for (int i = 0; i < C; ++i)
#pragma unroll
                        for (int i2 = 0; i2 < C; ++i2)
                            conflict |= sblk[t * C + i] == sblk[(pos + q) * C + i2];
                }
            }
            // First group that is inactive or conflicts ends the window.
            const uint64_t stop = __ballot(!active || conflict) & kGroupLsb;
            const uint32_t width = stop ? (uint32_t)(__builtin_ctzll(stop) >> 3) : 8u;
            if (g < width) {
                const uint64_t m = mask_word(smask, t, w);
                uint64_t B[C];
#pragma unroll
                for (int i = 0; i < C; ++i)
                    B[i] = __hip_atomic_load(&p.words[sblk[t * C + i] * 8 + w], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                const JA<C> ja = reduce_ja<C>(B, m);
                const int best = decide<C>(ja, s_rank);
                if (best >= 0) {
                    const uint64_t old = pick<C>(B, best);
                    if (m & ~old)
                        atomic_or_word(&p.words[sblk[t * C + best] * 8 + w], m);
                }
            }
            __builtin_amdgcn_s_waitcnt(0); // this window's atomics are done before the next reads
            pos += width;
        }
        wave_sync();
    }
}

__global__ void fill_zero_kernel(uint64_t *p, uint64_t n_words)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride)
        p[i] = 0;
}

// ------------------------------------------------------------ launchers

KParams make_kparams(const bbfc_filter &f)
{
    KParams p{};
    p.words = f.d_words;
    p.rank = f.d_rank;
    p.M = f.M;
    p.fm_magic = f.fm.magic;
    p.fm_sh1 = f.fm.sh1;
    p.fm_sh2 = f.fm.sh2;
    p.pow2_shift = f.pow2_shift;
    p.k = f.k;
    for (uint32_t i = 0; i < f.c; ++i)
        p.block_mult[i] = f.block_mult[i];
    for (uint32_t i = 0; i < f.k; ++i)
        p.bit_mult[i] = f.bit_mult[i];
    return p;
}

uint64_t insert_inflight(const bbfc_filter &f)
{
    uint64_t lim = f.max_inflight ? f.max_inflight : f.M / 32;
    return lim < (uint64_t)kTile ? (uint64_t)kTile : lim;
}

namespace {

// Resident wavefronts the device can hold for a kernel, as workgroups.
template <typename K>
uint64_t resident_wgs(K kernel, size_t dyn_lds, int num_cus)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWGSize, dyn_lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return (uint64_t)per_cu * (uint64_t)num_cus;
}

size_t rank_lds_bytes(const bbfc_filter &f)
{
    return f.c > 1 ? (size_t)(f.k + 1) * kRankStride * sizeof(uint16_t) : 0;
}

template <int C, int MODE>
hipError_t insert_impl(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    const uint64_t n_tiles = (n + kTile - 1) / kTile;
    const size_t lds = rank_lds_bytes(f);
    const uint64_t cap_waves = insert_inflight(f) / kTile;
    uint64_t wgs = resident_wgs(insert_kernel<C, MODE>, lds, f.num_cus);
    const uint64_t cap_wgs = (cap_waves + kWavesPerWG - 1) / kWavesPerWG;
    const uint64_t need = (n_tiles + kWavesPerWG - 1) / kWavesPerWG;
    wgs = wgs < cap_wgs ? wgs : cap_wgs;
    wgs = wgs < need ? wgs : need;
    if (wgs < 1)
        wgs = 1;
    hipLaunchKernelGGL((insert_kernel<C, MODE>), dim3((uint32_t)wgs), dim3(kWGSize), lds, s, make_kparams(f), keys,
                       n, n_tiles);
    return hipGetLastError();
}

template <int C, int MODE>
hipError_t insert_det_impl(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    const uint64_t n_tiles = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL((insert_det_kernel<C, MODE>), dim3(1), dim3(kWave), rank_lds_bytes(f), s, make_kparams(f),
                       keys, n, n_tiles);
    return hipGetLastError();
}

template <int C, int MODE, bool EARLY>
hipError_t query_launch(const bbfc_filter &f, const uint64_t *keys, uint64_t n, uint64_t *out, hipStream_t s)
{
    const uint64_t n_tiles = (n + kTile - 1) / kTile;
    uint64_t wgs = resident_wgs(query_kernel<C, MODE, EARLY>, 0, f.num_cus);
    const uint64_t need = (n_tiles + kWavesPerWG - 1) / kWavesPerWG;
    wgs = wgs < need ? wgs : need;
    if (wgs < 1)
        wgs = 1;
    hipLaunchKernelGGL((query_kernel<C, MODE, EARLY>), dim3((uint32_t)wgs), dim3(kWGSize), 0, s, make_kparams(f),
                       keys, n, out, n_tiles);
    return hipGetLastError();
}

template <int C, int MODE>
hipError_t query_impl(const bbfc_filter &f, const uint64_t *keys, uint64_t n, uint64_t *out, hipStream_t s)
{
    if (C > 1 && f.query_early_exit)
        return query_launch<C, MODE, true>(f, keys, n, out, s);
    return query_launch<C, MODE, false>(f, keys, n, out, s);
}

// Dispatch on (choices, hash mode) to a template instance.
template <template <int, int> class Op, typename... Args>
hipError_t dispatch(const bbfc_filter &f, Args... args)
{
#define BBFC_CASE(CC, MM)                                                                                              \
    if (f.c == CC && f.hash_mode == MM)                                                                               \
        return Op<CC, MM>::run(f, args...);
#define BBFC_MODES(CC) BBFC_CASE(CC, kModeOne) BBFC_CASE(CC, kModePow2) BBFC_CASE(CC, kModeEven) BBFC_CASE(CC, kModeOdd)
    BBFC_MODES(1)
    BBFC_MODES(2)
    BBFC_MODES(3)
    BBFC_MODES(4)
#undef BBFC_MODES
#undef BBFC_CASE
    return hipErrorInvalidValue;
}

template <int C, int M>
struct InsertOp {
    static hipError_t run(const bbfc_filter &f, const uint64_t *k, uint64_t n, hipStream_t s)
    {
        return insert_impl<C, M>(f, k, n, s);
    }
};
template <int C, int M>
struct InsertDetOp {
    static hipError_t run(const bbfc_filter &f, const uint64_t *k, uint64_t n, hipStream_t s)
    {
        return insert_det_impl<C, M>(f, k, n, s);
    }
};
template <int C, int M>
struct QueryOp {
    static hipError_t run(const bbfc_filter &f, const uint64_t *k, uint64_t n, uint64_t *o, hipStream_t s)
    {
        return query_impl<C, M>(f, k, n, o, s);
    }
};

} // namespace

hipError_t launch_insert(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    return dispatch<InsertOp>(f, keys, n, s);
}

hipError_t launch_insert_det(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    return dispatch<InsertDetOp>(f, keys, n, s);
}

hipError_t launch_query(const bbfc_filter &f, const uint64_t *keys, uint64_t n, uint64_t *out, hipStream_t s)
{
    return dispatch<QueryOp>(f, keys, n, out, s);
}

hipError_t launch_fill_zero(uint64_t *p, uint64_t n_words, hipStream_t s)
{
    uint64_t blocks = (n_words + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, n_words);
    return hipGetLastError();
}

} // namespace bbfc
