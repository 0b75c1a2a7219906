// Bulk insert for filters with sub-arrays (Section 3.4, Parallelization).
//
// The paper parallelises insertion by giving each thread a sub-array: a
// distributor routes every key to the sub-array h_0(x) and a single writer
// inserts it there. On the GPU the routing is a stable radix partition of the
// keys by h_0, and the single writer of a sub-array is one wavefront that
// stages the whole sub-array in LDS, inserts the sub-array's keys in their
// original order, and writes the sub-array back. Nothing touches HBM at
// random: the partition passes stream the keys, the insert streams the
// sorted keys and each sub-array once.
//
// The result equals inserting the keys one at a time in index order
// (Section 3.2 applied key by key): the partition is stable, so every
// sub-array sees its keys in index order, and inside a sub-array the
// wavefront decides a key only after every earlier key that shares one of
// its candidate blocks. A key's candidate blocks change only when a key that
// shares one of them is inserted, and such keys are decided before it if they
// come earlier and after it if later, so every key sees its candidates as in
// the one-at-a-time order. Keys decided in the same step share no candidate
// and are decided together.
//
// Kernels, per radix pass p (digits of h_0, least significant first):
//   bulk_hist_kernel     per group of up to 16 tiles of 4096 keys, the
//                        count of each digit
//   scan kernels         exclusive prefix over (digit, group), digit-major
//   bulk_scatter_kernel  one workgroup per group: stable scatter of each of
//                        its tiles in order, staged in LDS so the writes go
//                        out as runs
// then bulk_insert_kernel over the sorted keys. Counting per group rather
// than per tile keeps the count table (read and written with one 4-byte
// access per digit and group) small next to the keys.
#include <stdint.h>

#include <utility>

#include <hip/hip_runtime.h>

#include "bbfc_internal.hpp"
#include "bbfc_tile.hpp"

namespace bbfc {

namespace {

constexpr int kPartThreads = 256;
constexpr int kPartPerLane = 16;
constexpr int kPartTile = kPartThreads * kPartPerLane; // 4096 keys per tile
constexpr int kPartWaveKeys = kWave * kPartPerLane;    // 1024 keys per wavefront of a tile
constexpr uint32_t kMaxTilesPerGroup = 16; // counted groups: up to 16 tiles, at least ~2048 groups
constexpr int kMaxDigitBits = 9;
constexpr int kMaxDigits = 1 << kMaxDigitBits;
constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int kScanBlock = kScanThreads * kScanPerThread; // 4096 counts per scan block
constexpr int kScanTopThreads = 1024;
constexpr int kClaimSlots = 256;                          // hashed claim table entries per wavefront
constexpr int kBulkSlotDw = 16;                           // LDS dwords per key mask in the bulk insert

// One radix digit of h_0: (h_0(x) >> shift) & mask; MODE is the hash mode
// of the number of sub-arrays, fixed per launch.
struct Digit {
    HashMod sub;
    uint64_t sub_mult;
    uint32_t shift;
    uint32_t mask;
    template <int MODE>
    __device__ __forceinline__ uint32_t of(uint64_t x) const
    {
        return (uint32_t)(hash_mod<MODE>(sub, sub_mult, x) >> shift) & mask;
    }
};

// f(integral_constant<int, R>) for R = 0..N-1, so array indices stay
// compile-time constants however large the body.
template <typename F, int... R>
__device__ __forceinline__ void static_for(F &&f, std::integer_sequence<int, R...>)
{
    (f(std::integral_constant<int, R>{}), ...);
}

__device__ __forceinline__ uint64_t lanemask_lt(uint32_t lane)
{
    return lane == 0 ? 0 : (~0ull >> (64 - lane));
}

// Set bits of m below bit `lane`.
__device__ __forceinline__ uint32_t count_below(uint64_t m, uint32_t lane)
{
    return (uint32_t)__popcll(m & lanemask_lt(lane));
}

// v / D for v < 48 (D = 3) or v < 56 (D = 7), with a 24-bit multiply.
template <int D>
__device__ __forceinline__ uint32_t div_by(uint32_t v)
{
    static_assert(D == 3 || D == 7, "divisor 3 or 7");
    if constexpr (D == 3)
        return (v * 43u) >> 7;
    else
        return (v * 37u) >> 8;
}

// The value of the first lane of each aligned group of LPK (4 or 8) lanes.
template <int LPK>
__device__ __forceinline__ uint32_t group_first(uint32_t v)
{
    static_assert(LPK == 4 || LPK == 8, "groups of 4 or 8 lanes");
    if constexpr (LPK == 4)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x00, 0xF, 0xF, false); // quad_perm 0,0,0,0
    else
        return (uint32_t)__shfl((int)v, (int)(__lane_id() & ~7u));
}

// ----------------------------------------------------------- partition

template <int MODE>
__global__ __launch_bounds__(kPartThreads) void bulk_hist_kernel(const uint64_t *__restrict__ keys, uint64_t n,
                                                                 Digit dg, uint32_t n_digits,
                                                                 uint32_t *__restrict__ counts, uint32_t n_groups,
                                                                 uint32_t tiles_per_group)
{
    __shared__ uint32_t h[kMaxDigits];
    for (uint32_t i = threadIdx.x; i < n_digits; i += kPartThreads)
        h[i] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * tiles_per_group * kPartTile;
    const uint32_t rounds = kPartPerLane * tiles_per_group;
#pragma unroll 8
    for (uint32_t r = 0; r < rounds; ++r) {
        const uint64_t idx = base + (uint64_t)r * kPartThreads + threadIdx.x;
        if (idx < n)
            atomicAdd(&h[dg.of<MODE>(keys[idx])], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_digits; i += kPartThreads)
        counts[(uint64_t)i * n_groups + blockIdx.x] = h[i];
}

// Exclusive scan of uint32 counts in three launches: block sums, a scan of
// the block sums in one workgroup, then each block rescanned with its offset.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    // Hillis-Steele over the workgroup in LDS (blockDim.x entries).
    const uint32_t t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (uint32_t off = 1; off < blockDim.x; off <<= 1) {
        const uint32_t add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const uint32_t incl = sh[t];
    total = sh[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t *__restrict__ in, uint64_t len,
                                                                   uint32_t *__restrict__ partial)
{
    __shared__ uint32_t sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
    for (int r = 0; r < kScanPerThread; ++r) {
        const uint64_t i = base + (uint64_t)r * kScanThreads + threadIdx.x;
        if (i < len)
            s += in[i];
    }
    uint32_t total;
    (void)block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = total;
}

// One workgroup: exclusive scan of n_part block sums in place.
__global__ __launch_bounds__(kScanTopThreads) void scan_partials_kernel(uint32_t *__restrict__ partial,
                                                                        uint32_t n_part)
{
    __shared__ uint32_t sh[kScanTopThreads];
    const uint32_t per = (n_part + kScanTopThreads - 1) / kScanTopThreads;
    const uint32_t lo = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t i = lo; i < lo + per && i < n_part; ++i)
        s += partial[i];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, total);
    for (uint32_t i = lo; i < lo + per && i < n_part; ++i) {
        const uint32_t v = partial[i];
        partial[i] = run;
        run += v;
    }
}

// Each thread owns kScanPerThread consecutive counts of the block.
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(uint32_t *__restrict__ data, uint64_t len,
                                                                  const uint32_t *__restrict__ partial)
{
    __shared__ uint32_t sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanPerThread;
    uint32_t v[kScanPerThread];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanPerThread; ++r) {
        v[r] = base + r < len ? data[base + r] : 0;
        s += v[r];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, total) + partial[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kScanPerThread; ++r) {
        if (base + r < len)
            data[base + r] = run;
        run += v[r];
    }
}

// Stable scatter of one group of tiles, tile after tile. The scan gives the
// group's run start for each digit; each tile takes the current start and
// moves it past its own keys of that digit. Inside a tile, wavefront w owns
// the keys [w*1024, (w+1)*1024), lane l round r takes key w*1024 + 64r + l,
// so key order is (w, r, l). 1) per-wavefront digit counts; 2) where each
// (wavefront, digit) run starts inside the tile's staging area; 3) every
// round ranks its keys among equal digits of the round (ballot matching)
// and stages them; 4) the staged tile, now ordered by digit, is written to
// the tile's digit runs.
template <int MODE>
__global__ __launch_bounds__(kPartThreads) void bulk_scatter_kernel(const uint64_t *__restrict__ in,
                                                                    uint64_t *__restrict__ out, uint64_t n, Digit dg,
                                                                    uint32_t n_digits,
                                                                    const uint32_t *__restrict__ offsets,
                                                                    uint32_t n_groups, uint32_t tiles_per_group)
{
    extern __shared__ uint64_t staged[]; // kPartTile keys
    __shared__ uint32_t wcnt[kPartThreads / kWave][kMaxDigits];
    __shared__ uint32_t tpre[kMaxDigits]; // digit run start inside the tile
    __shared__ uint32_t gofs[kMaxDigits]; // digit run start in the output
    __shared__ uint32_t scan_sh[kPartThreads];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t w = threadIdx.x / kWave;
    // thread t owns digits t and t + 256: its running output position for each
    uint32_t run_at[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t d = threadIdx.x + h * kPartThreads;
        if (d < n_digits)
            run_at[h] = offsets[(uint64_t)d * n_groups + blockIdx.x];
    }
    for (uint32_t tg = 0; tg < tiles_per_group; ++tg) {
        const uint64_t tile_base = ((uint64_t)blockIdx.x * tiles_per_group + tg) * kPartTile;
        if (tile_base >= n)
            break;
        const uint64_t wave_base = tile_base + (uint64_t)w * kPartWaveKeys;

        uint64_t key[kPartPerLane];
#pragma unroll
        for (int r = 0; r < kPartPerLane; ++r) {
            const uint64_t idx = wave_base + (uint64_t)r * kWave + lane;
            key[r] = idx < n ? in[idx] : 0;
        }
        for (uint32_t d = lane; d < n_digits; d += kWave)
            wcnt[w][d] = 0;
        wave_sync();
#pragma unroll
        for (int r = 0; r < kPartPerLane; ++r) {
            const uint64_t idx = wave_base + (uint64_t)r * kWave + lane;
            if (idx < n)
                atomicAdd(&wcnt[w][dg.of<MODE>(key[r])], 1u);
        }
        __syncthreads();

        // digit totals of the tile, their exclusive prefix, and the per-wavefront
        // run starts (digits d = t and t + 256 for thread t)
        uint32_t tot[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t d = threadIdx.x + h * kPartThreads;
            if (d < n_digits)
                for (int ww = 0; ww < kPartThreads / kWave; ++ww)
                    tot[h] += wcnt[ww][d];
        }
        uint32_t total0;
        const uint32_t pre0 = block_exclusive_scan(tot[0], scan_sh, total0);
        uint32_t total1;
        const uint32_t pre1 = block_exclusive_scan(tot[1], scan_sh, total1) + total0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t d = threadIdx.x + h * kPartThreads;
            if (d < n_digits) {
                uint32_t run = h == 0 ? pre0 : pre1;
                tpre[d] = run;
                gofs[d] = run_at[h];
                run_at[h] += tot[h];
                for (int ww = 0; ww < kPartThreads / kWave; ++ww) {
                    const uint32_t c = wcnt[ww][d];
                    wcnt[ww][d] = run;
                    run += c;
                }
            }
        }
        __syncthreads();

        static_for(
            [&](auto rc) __attribute__((always_inline)) {
                constexpr int r = decltype(rc)::value;
                const uint64_t idx = wave_base + (uint64_t)r * kWave + lane;
                const bool valid = idx < n;
                const uint32_t d = valid ? dg.of<MODE>(key[r]) : 0;
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int b = 0; b < kMaxDigitBits; ++b) { // bits above the digit are zero in every lane
                    const uint64_t m = __ballot((d >> b) & 1);
                    peers &= ((d >> b) & 1) ? m : ~m;
                }
                if (valid) {
                    const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt(lane));
                    const uint32_t pos = wcnt[w][d] + rank;
                    staged[pos] = key[r];
                }
                wave_sync(); // every lane has read its run start before the leader moves it
                if (valid && (peers & lanemask_lt(lane)) == 0)
                    wcnt[w][d] += (uint32_t)__popcll(peers);
                wave_sync();
            },
            std::make_integer_sequence<int, kPartPerLane>{});
        __syncthreads();

        const uint64_t left = n - tile_base;
        const uint32_t in_tile = left < (uint64_t)kPartTile ? (uint32_t)left : (uint32_t)kPartTile;
        for (uint32_t i = threadIdx.x; i < in_tile; i += kPartThreads) {
            const uint64_t x = staged[i];
            const uint32_t d = dg.of<MODE>(x);
            const uint64_t at = (uint64_t)gofs[d] + (uint32_t)(i - tpre[d]);
            if (at < n) // always true for consistent counts; keeps a stray index inside the buffer
                out[at] = x;
        }
        __syncthreads(); // the next tile reuses the staging, counts and run starts
    }
}

// --------------------------------------------------------------- insert

// LDS of one wavefront of the insert kernel. Every byte counts: the
// wavefronts that fit in a CU's LDS next to the rank table set how much
// latency is hidden (at k = 11 and S = 256: seven).
template <int SUB, int C>
struct WaveLds {
    static constexpr size_t kSub = (size_t)SUB * 64;                    // the staged sub-array
    static constexpr size_t kSlots = (size_t)kTile * kBulkSlotDw * 4;   // key masks
    static constexpr size_t kClaim = (size_t)kClaimSlots * 4;          // claim bits of 32 lanes
    static constexpr size_t kBytes = kSub + kSlots + kClaim;
};

// Lane src's 64-bit value.
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Each wavefront takes the sub-arrays whose run of sorted keys starts in its
// share [c0, c1) of the positions, and for each: stages the sub-array in
// LDS, inserts the run's keys in steps of keys with disjoint candidates
// (each after the earlier keys it conflicts with), and writes the sub-array
// back. S <= SUB blocks per sub-array.
template <int C, int SUB>
__global__ __launch_bounds__(512) void bulk_insert_kernel(KParams p, const uint64_t *__restrict__ sorted, uint64_t n,
                                                           uint32_t waves_per_wg, uint64_t n_waves)
{
    using WL = WaveLds<SUB, C>;
    // Four lanes per key, two block words each: a step decides up to 16
    // keys. Measured on 2^30 keys with 256 blocks per sub-array, this beats
    // eight lanes per key (steps of 8 keys) and two (each lane reduces four
    // words).
    constexpr int LPK = 4;
    constexpr int KW = 8 / LPK;      // words per lane
    constexpr int KPR = kWave / LPK; // keys per step
    extern __shared__ __align__(16) uint8_t lds[];
    uint16_t *s_rank = reinterpret_cast<uint16_t *>(lds);
    const size_t rank_bytes = C > 1 ? (((size_t)(p.k + 1) * kRankStride * 2 + 15) & ~(size_t)15) : 0;
    if constexpr (C > 1) {
        const uint32_t nr = (p.k + 1) * kRankStride;
        for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x)
            s_rank[i] = p.rank[i];
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    uint8_t *mine = lds + rank_bytes + (size_t)wv * WL::kBytes;
    uint64_t *sub = reinterpret_cast<uint64_t *>(mine);
    uint32_t *smask = reinterpret_cast<uint32_t *>(mine + WL::kSub);
    uint32_t *claim = reinterpret_cast<uint32_t *>(mine + WL::kSub + WL::kSlots);
    for (int i = lane; i < kClaimSlots; i += kWave)
        claim[i] = 0;

    const uint64_t S = p.blk.b;
    const uint64_t gw = (uint64_t)blockIdx.x * waves_per_wg + wv;
    const uint64_t c0 = n * gw / n_waves;
    const uint64_t c1 = n * (gw + 1) / n_waves;
    auto h0 = [&](uint64_t x) { return hash_mod_rt(p.sub, p.sub_mult, x); };

    uint64_t pos = c0;
    if (pos > 0 && pos < c1) {
        // the run of the sub-array that started before c0 belongs to the previous share
        const uint64_t prev = h0(sorted[pos - 1]);
        for (;;) {
            const uint64_t idx = pos + lane;
            const bool same = idx < n && h0(sorted[idx]) == prev;
            const uint64_t b = __ballot(same);
            const uint32_t cnt = (uint32_t)__popcll(b); // the equal keys form a prefix of the lanes
            pos += cnt;
            if (cnt < kWave)
                break;
        }
    }

    const uint32_t g = lane / LPK;
    const uint32_t w0 = (lane % LPK) * KW;
    constexpr int kSubIters = SUB * 8 / (2 * kWave); // 16-byte pieces per lane of a staged sub-array
    constexpr int kBatch = kSubIters < 8 ? kSubIters : 8;
    const uint64_t n_words = S * 8;
    uint64_t v = pos < c1 ? uniform_u64(h0(sorted[pos])) : 0;
    while (pos < c1) {
        // stage sub-array v; its first chunk of keys is loaded alongside
        uint64_t *gsub = p.words + v * S * 8;
        uint64_t x = pos + lane < n ? sorted[pos + lane] : 0;
#pragma unroll
        for (int b0 = 0; b0 < kSubIters; b0 += kBatch) {
            ulonglong2 t[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint64_t i = (uint64_t)(b0 + b) * 2 * kWave + lane * 2;
                t[b] = i < n_words ? *reinterpret_cast<const ulonglong2 *>(gsub + i) : make_ulonglong2(0, 0);
            }
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint64_t i = (uint64_t)(b0 + b) * 2 * kWave + lane * 2;
                if (i < n_words) {
                    sub[i] = t[b].x;
                    sub[i + 1] = t[b].y;
                }
            }
        }
        wave_sync();

        uint64_t v_next = 0;
        bool v_next_known = false;
        for (;;) {
            const bool valid = pos + lane < n && h0(x) == v;
            const uint64_t vb = __ballot(valid);
            const uint32_t n_valid = (uint32_t)__popcll(vb); // a prefix of the lanes
            if (n_valid == 0)
                break;
            if (n_valid < (uint32_t)kWave && pos + n_valid < n) {
                // lane n_valid holds the first key of the next sub-array's run
                v_next = uniform_u64(shfl_u64(h0(x), (int)n_valid));
                v_next_known = true;
            }

            // key masks into LDS slots, candidate blocks (inside the sub-array) in registers
            uint32_t *slot = smask + lane * kBulkSlotDw;
#pragma unroll
            for (int d = 0; d < 16; d += 2)
                *reinterpret_cast<uint2 *>(slot + d) = make_uint2(0, 0);
            wave_sync();
            auto set_bit = [slot](uint32_t f) { atomicOr(slot + (f >> 5), 1u << (f & 31)); };
            if (valid) {
                if (p.distinct)
                    distinct_bits(p.bit_mult, p.k, x, set_bit);
                else
                    random_bits(p.bit_mult, p.k, x, set_bit);
            }
            uint32_t cand[C];
#pragma unroll
            for (int i = 0; i < C; ++i)
                cand[i] = (uint32_t)hash_mod_rt(p.blk, p.block_mult[i], x);

            // the next chunk's keys are in flight while this chunk is inserted
            // (issued after the last use of x, so waiting for x does not wait for them)
            const uint64_t nidx = pos + kWave + lane;
            const bool more = n_valid == (uint32_t)kWave;
            const uint64_t x_next = more && nidx < n ? sorted[nidx] : 0;

            // P: the earlier keys of the chunk that share a candidate (claim
            // bits hashed into kClaimSlots 32-bit entries; a collision only
            // adds a dependency). The lower half claims first and both halves
            // read; then the upper half claims and reads.
            uint64_t P = 0;
#pragma unroll
            for (uint32_t half = 0; half < 2; ++half) {
                const bool mine_half = (lane >> 5) == half;
                if (valid && mine_half) {
#pragma unroll
                    for (int i = 0; i < C; ++i)
                        atomicOr(&claim[cand[i] % kClaimSlots], 1u << (lane & 31));
                }
                wave_sync();
                if ((lane >> 5) >= half) {
                    uint32_t q = 0;
#pragma unroll
                    for (int i = 0; i < C; ++i)
                        q |= claim[cand[i] % kClaimSlots];
                    P |= (uint64_t)q << (32 * half);
                }
                wave_sync();
                if (valid && mine_half) {
#pragma unroll
                    for (int i = 0; i < C; ++i)
                        claim[cand[i] % kClaimSlots] = 0;
                }
                wave_sync();
            }
            P &= lanemask_lt(lane);

            // Steps: each takes the first KPR pending keys whose earlier
            // conflicting keys are all done. The keys of a step share no
            // candidate, and every key is decided after each earlier key
            // that shares one, so the result is the sequential one. The
            // lowest pending key is always ready: at most 64 steps.
            uint64_t done = 0;
            while (done != vb) {
                const bool ready = valid && !((done >> lane) & 1) && (P & ~done) == 0;
                const uint64_t rb = __ballot(ready);
                const bool take = ready && count_below(rb, lane) < (uint32_t)KPR;
                const uint64_t tb = __ballot(take);
                const uint32_t cnt = (uint32_t)__popcll(tb);
                // taken key number r goes to lane LPK*r; the other lanes fill the
                // remaining lanes in order, so that the push is a permutation
                const uint32_t tr = count_below(tb, lane);
                uint32_t dest;
                if (take) {
                    dest = LPK * tr;
                } else {
                    const uint32_t nr = lane - tr;
                    const uint32_t gap = (LPK - 1) * cnt;
                    dest = nr < gap ? LPK * div_by<LPK - 1>(nr) + 1 + (nr - (LPK - 1) * div_by<LPK - 1>(nr))
                                    : LPK * cnt + (nr - gap);
                }
                const int daddr = (int)(dest * 4);
                uint32_t rc[C];
#pragma unroll
                for (int i = 0; i < C; ++i)
                    rc[i] = group_first<LPK>((uint32_t)__builtin_amdgcn_ds_permute(daddr, (int)cand[i]));
                const uint32_t src = group_first<LPK>((uint32_t)__builtin_amdgcn_ds_permute(daddr, (int)lane));
                const bool active = g < cnt;
                uint64_t mw[KW];
                const uint32_t *ks = smask + src * kBulkSlotDw + 2 * w0;
#pragma unroll
                for (int q = 0; q < KW; ++q)
                    mw[q] = *reinterpret_cast<const uint64_t *>(ks + 2 * q);
                uint64_t B[C][KW];
#pragma unroll
                for (int i = 0; i < C; ++i)
#pragma unroll
                    for (int q = 0; q < KW; ++q)
                        B[i][q] = sub[(uint64_t)rc[i] * 8 + w0 + q];
                const JA<C> ja = reduce_ja<C, LPK, KW>(B, mw);
                const int best = decide<C>(ja, s_rank);
                if (active && best >= 0) {
                    uint32_t blk = rc[0];
#pragma unroll
                    for (int i = 1; i < C; ++i)
                        blk = best == i ? rc[i] : blk;
#pragma unroll
                    for (int q = 0; q < KW; ++q) {
                        const uint64_t old = pick<C, KW>(B, best, q);
                        if (mw[q] & ~old)
                            sub[(uint64_t)blk * 8 + w0 + q] = old | mw[q];
                    }
                }
                wave_sync();
                done |= tb;
            }
            pos += n_valid;
            if (!more)
                break;
            x = x_next;
        }

        wave_sync();
#pragma unroll
        for (int b = 0; b < kSubIters; ++b) {
            const uint64_t i = (uint64_t)b * 2 * kWave + lane * 2;
            if (i < n_words) {
                ulonglong2 t;
                t.x = sub[i];
                t.y = sub[i + 1];
                *reinterpret_cast<ulonglong2 *>(gsub + i) = t;
            }
        }
        wave_sync();
        if (pos >= c1 || pos >= n)
            break;
        v = v_next_known ? v_next : uniform_u64(h0(sorted[pos]));
    }
}

// ------------------------------------------------------------- planning

struct Plan {
    uint32_t passes = 0;
    uint32_t bits[3] = {0, 0, 0};
    uint32_t tiles_per_group = 1;
    uint64_t n_groups = 0;   // groups of tiles_per_group tiles (the counted unit)
    uint64_t counts_len = 0; // max over passes of n_digits * n_groups
    uint64_t n_scan_blocks = 0;
    int sub_max = 0;         // LDS sub-array capacity in blocks
    // workspace layout (bytes, 256-aligned)
    uint64_t off_keys_a = 0, off_keys_b = 0, off_counts = 0, off_partial = 0, bytes = 0;
};

uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

int sub_capacity(uint64_t S)
{
    if (S <= 256)
        return 256;
    if (S <= 512)
        return 512;
    if (S <= 1024)
        return 1024;
    return 0;
}

Plan make_plan(const bbfc_filter &f, uint64_t n)
{
    Plan pl;
    uint32_t tbits = 0;
    while (tbits < 64 && ((uint64_t)1 << tbits) < f.T)
        ++tbits;
    pl.passes = (tbits + kMaxDigitBits - 1) / kMaxDigitBits;
    for (uint32_t q = 0; q < pl.passes; ++q) { // spread the bits evenly over the passes
        pl.bits[q] = tbits / pl.passes + (q < tbits % pl.passes ? 1 : 0);
    }
    const uint64_t n_tiles = (n + kPartTile - 1) / kPartTile;
    const uint64_t tpg = n_tiles / 2048;
    pl.tiles_per_group = tpg < 1 ? 1 : (tpg > kMaxTilesPerGroup ? kMaxTilesPerGroup : (uint32_t)tpg);
    pl.n_groups = (n_tiles + pl.tiles_per_group - 1) / pl.tiles_per_group;
    uint32_t max_bits = 0;
    for (uint32_t q = 0; q < pl.passes; ++q)
        max_bits = pl.bits[q] > max_bits ? pl.bits[q] : max_bits;
    pl.counts_len = ((uint64_t)1 << max_bits) * pl.n_groups;
    pl.n_scan_blocks = (pl.counts_len + kScanBlock - 1) / kScanBlock;
    pl.sub_max = sub_capacity(f.S);
    uint64_t at = 0;
    if (pl.passes >= 1) {
        pl.off_keys_a = at;
        at = align256(at + n * 8);
    }
    if (pl.passes >= 2) {
        pl.off_keys_b = at;
        at = align256(at + n * 8);
    }
    if (pl.passes >= 1) {
        pl.off_counts = at;
        at = align256(at + pl.counts_len * 4);
        pl.off_partial = at;
        at = align256(at + pl.n_scan_blocks * 4);
    }
    pl.bytes = at;
    return pl;
}

template <int C, int SUB>
size_t insert_lds_bytes(uint32_t k, uint32_t waves)
{
    const size_t rank = C > 1 ? (((size_t)(k + 1) * kRankStride * 2 + 15) & ~(size_t)15) : 0;
    return rank + (size_t)waves * WaveLds<SUB, C>::kBytes;
}

template <int C, int SUB>
hipError_t launch_insert_sub(const bbfc_filter &f, const uint64_t *sorted, uint64_t n, hipStream_t s)
{
    const size_t per = WaveLds<SUB, C>::kBytes;
    const size_t rank = insert_lds_bytes<C, SUB>(f.k, 0);
    if (f.max_lds < rank + per)
        return hipErrorInvalidValue;
    uint32_t waves = (uint32_t)((f.max_lds - rank) / per);
    if (waves > 8) // the kernel's launch bound: 512 threads
        waves = 8;
    const size_t lds = rank + waves * per;
    // one workgroup per CU: the LDS holds `waves` sub-arrays at a time
    uint64_t wgs = (uint64_t)(f.num_cus > 0 ? f.num_cus : 256);
    const uint64_t n_waves = wgs * waves;
    hipError_t e = hipFuncSetAttribute((const void *)bulk_insert_kernel<C, SUB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((bulk_insert_kernel<C, SUB>), dim3((uint32_t)wgs), dim3(waves * kWave), lds, s,
                       make_kparams(f), sorted, n, waves, n_waves);
    return hipGetLastError();
}

template <int C>
hipError_t launch_insert_c(const bbfc_filter &f, int sub_max, const uint64_t *sorted, uint64_t n, hipStream_t s)
{
    switch (sub_max) {
    case 256:
        return launch_insert_sub<C, 256>(f, sorted, n, s);
    case 512:
        return launch_insert_sub<C, 512>(f, sorted, n, s);
    default:
        return launch_insert_sub<C, 1024>(f, sorted, n, s);
    }
}

template <int MODE>
hipError_t launch_hist_m(uint32_t n_groups, uint32_t tpg, hipStream_t s, const uint64_t *src, uint64_t n, const Digit &dg,
                         uint32_t n_digits, uint32_t *counts)
{
    hipLaunchKernelGGL(bulk_hist_kernel<MODE>, dim3(n_groups), dim3(kPartThreads), 0, s, src, n, dg, n_digits, counts,
                       n_groups, tpg);
    return hipGetLastError();
}

hipError_t launch_hist(uint32_t mode, uint32_t n_groups, uint32_t tpg, hipStream_t s, const uint64_t *src, uint64_t n,
                       const Digit &dg, uint32_t n_digits, uint32_t *counts)
{
    switch (mode) {
    case kModePow2:
        return launch_hist_m<kModePow2>(n_groups, tpg, s, src, n, dg, n_digits, counts);
    case kModeEven:
        return launch_hist_m<kModeEven>(n_groups, tpg, s, src, n, dg, n_digits, counts);
    default:
        return launch_hist_m<kModeOdd>(n_groups, tpg, s, src, n, dg, n_digits, counts);
    }
}

template <int MODE>
hipError_t launch_scatter_m(uint32_t n_groups, uint32_t tpg, hipStream_t s, const uint64_t *src, uint64_t *dst, uint64_t n,
                            const Digit &dg, uint32_t n_digits, const uint32_t *offsets)
{
    hipError_t e = hipFuncSetAttribute((const void *)bulk_scatter_kernel<MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kPartTile * 8);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(bulk_scatter_kernel<MODE>, dim3(n_groups), dim3(kPartThreads), kPartTile * 8, s, src, dst, n,
                       dg, n_digits, offsets, n_groups, tpg);
    return hipGetLastError();
}

// Radix passes run only with T > 1 sub-arrays, so the mode of T is never One.
hipError_t launch_scatter(uint32_t mode, uint32_t n_groups, uint32_t tpg, hipStream_t s, const uint64_t *src, uint64_t *dst,
                          uint64_t n, const Digit &dg, uint32_t n_digits, const uint32_t *offsets)
{
    switch (mode) {
    case kModePow2:
        return launch_scatter_m<kModePow2>(n_groups, tpg, s, src, dst, n, dg, n_digits, offsets);
    case kModeEven:
        return launch_scatter_m<kModeEven>(n_groups, tpg, s, src, dst, n, dg, n_digits, offsets);
    default:
        return launch_scatter_m<kModeOdd>(n_groups, tpg, s, src, dst, n, dg, n_digits, offsets);
    }
}

} // namespace

uint64_t bulk_workspace_bytes(const bbfc_filter &f, uint64_t n)
{
    return make_plan(f, n).bytes;
}

bool bulk_supported(const bbfc_filter &f)
{
    return sub_capacity(f.S) != 0 && make_plan(f, 1).passes <= 3;
}

hipError_t launch_bulk_insert(const bbfc_filter &f, const uint64_t *keys, uint64_t n, void *workspace,
                              hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const Plan pl = make_plan(f, n);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    uint64_t *bufs[2] = {reinterpret_cast<uint64_t *>(ws + pl.off_keys_a),
                         reinterpret_cast<uint64_t *>(ws + pl.off_keys_b)};
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + pl.off_counts);
    uint32_t *partial = reinterpret_cast<uint32_t *>(ws + pl.off_partial);
    const uint64_t *src = keys;
    uint32_t shift = 0;
    for (uint32_t q = 0; q < pl.passes; ++q) {
        Digit dg;
        dg.sub = f.sub;
        dg.sub_mult = f.sub_mult;
        dg.shift = shift;
        dg.mask = (1u << pl.bits[q]) - 1;
        const uint32_t n_digits = 1u << pl.bits[q];
        const uint64_t len = (uint64_t)n_digits * pl.n_groups;
        const uint64_t n_blocks = (len + kScanBlock - 1) / kScanBlock;
        uint64_t *dst = bufs[q & 1];
        hipError_t e = launch_hist(f.sub.mode, (uint32_t)pl.n_groups, pl.tiles_per_group, s, src, n, dg, n_digits,
                                   counts);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(scan_reduce_kernel, dim3((uint32_t)n_blocks), dim3(kScanThreads), 0, s, counts, len,
                           partial);
        hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanTopThreads), 0, s, partial,
                           (uint32_t)n_blocks);
        hipLaunchKernelGGL(scan_apply_kernel, dim3((uint32_t)n_blocks), dim3(kScanThreads), 0, s, counts, len,
                           partial);
        e = launch_scatter(f.sub.mode, (uint32_t)pl.n_groups, pl.tiles_per_group, s, src, dst, n, dg, n_digits,
                           counts);
        if (e != hipSuccess)
            return e;
        src = dst;
        shift += pl.bits[q];
    }
    switch (f.c) {
    case 1:
        return launch_insert_c<1>(f, pl.sub_max, src, n, s);
    case 2:
        return launch_insert_c<2>(f, pl.sub_max, src, n, s);
    case 3:
        return launch_insert_c<3>(f, pl.sub_max, src, n, s);
    default:
        return launch_insert_c<4>(f, pl.sub_max, src, n, s);
    }
}

} // namespace bbfc
