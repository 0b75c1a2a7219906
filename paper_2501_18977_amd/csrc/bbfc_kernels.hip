// Single-filter insert and query kernels for gfx950 and their launchers.
// The per-tile work (phase A hashing into LDS, phase B gathers, reductions,
// decisions, atomic writes) lives in bbfc_tile.hpp; these kernels hand tiles
// of one filter to resident wavefronts.
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include <hip/hip_runtime.h>

#include "bbfc_common.hpp"
#include "bbfc_internal.hpp"
#include "bbfc_tile.hpp"

namespace bbfc {

constexpr int kWavesPerWG = 4;
constexpr int kWGSize = kWave * kWavesPerWG;

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

// Unit u = tiles u*T .. u*T+T-1; units are strided over the wavefronts.
// Src: where key t comes from (an array, or a k-mer of a packed sequence).
template <int C, int LPK, int T, bool EARLY, typename Src>
__global__ __launch_bounds__(kWGSize) void query_kernel(KParams p, Src keys, uint64_t n, uint64_t *__restrict__ out,
                                                        uint64_t n_units)
{
    __shared__ uint32_t s_mask[kWavesPerWG][T * kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][T * kTile * C];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerWG;
    for (uint64_t u = (uint64_t)blockIdx.x * kWavesPerWG + wv; u < n_units; u += n_waves)
        query_tiles<C, LPK, T, EARLY>(p, keys, n, u * T * kTile, out + u * T, lane, s_mask[wv], s_blk[wv]);
}

// A query over several key arrays of one filter (a batch of requests that
// live in device memory): units are numbered piece after piece and each
// wavefront takes one contiguous run of them. The pieces' first units are
// staged in LDS; a binary search there finds the piece of a wavefront's first
// unit, and a cursor that only moves forward (about one step per piece of
// the run) finds the rest.
template <int C, int LPK, int T, bool EARLY>
__global__ __launch_bounds__(kWGSize) void query_pieces_kernel(KParams p, const QueryPiece *__restrict__ pieces,
                                                               uint32_t n_pieces, uint64_t n_units)
{
    __shared__ uint32_t s_mask[kWavesPerWG][T * kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][T * kTile * C];
    __shared__ uint32_t s_first[kMaxQueryPieces];
    for (uint32_t i = threadIdx.x; i < n_pieces; i += blockDim.x)
        s_first[i] = (uint32_t)pieces[i].unit_off;
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerWG;
    const uint64_t per = (n_units + n_waves - 1) / n_waves;
    const uint64_t u0 = ((uint64_t)blockIdx.x * kWavesPerWG + wv) * per;
    const uint64_t u1 = u0 + per < n_units ? u0 + per : n_units;
    if (u0 >= u1)
        return;
    // the last piece whose first unit is <= u0 (s_first[0] == 0)
    uint32_t f = 0, hi = n_pieces - 1;
    while (f < hi) {
        const uint32_t mid = (f + hi + 1) / 2;
        if (s_first[mid] <= u0)
            f = mid;
        else
            hi = mid - 1;
    }
    for (uint64_t u = u0; u < u1; ++u) {
        while (f + 1 < n_pieces && s_first[f + 1] <= u)
            ++f;
        const QueryPiece pc = pieces[f];
        const uint64_t lu = u - pc.unit_off;
        query_tiles<C, LPK, T, EARLY>(p, ArrayKeys{pc.keys}, pc.n, lu * T * kTile, pc.out + lu * T, lane, s_mask[wv],
                                      s_blk[wv]);
    }
}

template <int C, int LPK, int T, typename Src>
__global__ __launch_bounds__(kWGSize) void insert_kernel(KParams p, Src keys, uint64_t n, uint64_t n_units,
                                                         uint64_t n_waves)
{
    __shared__ uint32_t s_mask[kWavesPerWG][T * kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][T * kTile * C];
    extern __shared__ uint16_t s_rank[];
    load_rank_table<C>(p, s_rank);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    // n_waves <= the grid's wavefronts: the ones past it idle, which bounds
    // the keys in flight to n_waves * T * 64 exactly
    const uint64_t first = (uint64_t)blockIdx.x * kWavesPerWG + wv;
    for (uint64_t u = first < n_waves ? first : n_units; u < n_units; u += n_waves)
        insert_tiles<C, LPK, T>(p, s_rank, keys, n, u * T * kTile, lane, s_mask[wv], s_blk[wv]);
}

// Racing insert in tiles of 8 keys (insert_narrow_tile), for bounds on the
// keys in flight that leave the GPU mostly idle; n_waves as in insert_kernel.
template <int C, typename Src, bool REC>
__global__ __launch_bounds__(kWGSize) void insert_narrow_kernel(KParams p, Src keys, uint64_t n, uint64_t n_units,
                                                                uint64_t n_waves, uint8_t *__restrict__ rec)
{
    __shared__ uint32_t s_mask[kWavesPerWG][kNarrowKeys * kSlotDw];
    extern __shared__ uint16_t s_rank[];
    load_rank_table<C>(p, s_rank);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    // multipliers of f_(8j + l) for this lane's l, selected with constant
    // indices so that they stay in registers
    const uint32_t l = lane % 8;
    uint64_t am[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < (int)BBFC_MAX_BITS_PER_KEY; ++i)
        if ((uint32_t)(i % 8) == l)
            am[i / 8] = p.bit_mult[i];
    const uint64_t first = (uint64_t)blockIdx.x * kWavesPerWG + wv;
    for (uint64_t u = first < n_waves ? first : n_units; u < n_units; u += n_waves)
        insert_narrow_tile<C, Src, REC>(p, s_rank, keys, n, u * kNarrowKeys, lane, am, s_mask[wv], rec);
}

// insert_kernel that also writes each key's decision to rec[t] (see
// insert_tiles): a checking aid with the same schedule, never the timed kernel.
template <int C, int LPK, int T, typename Src>
__global__ __launch_bounds__(kWGSize) void insert_recorded_kernel(KParams p, Src keys, uint64_t n, uint64_t n_units,
                                                                  uint64_t n_waves, uint8_t *__restrict__ rec)
{
    __shared__ uint32_t s_mask[kWavesPerWG][T * kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][T * kTile * C];
    extern __shared__ uint16_t s_rank[];
    load_rank_table<C>(p, s_rank);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t first = (uint64_t)blockIdx.x * kWavesPerWG + wv;
    for (uint64_t u = first < n_waves ? first : n_units; u < n_units; u += n_waves)
        insert_tiles<C, LPK, T, Src, true>(p, s_rank, keys, n, u * T * kTile, lane, s_mask[wv], s_blk[wv], rec);
}

__global__ void fill_zero_kernel(uint64_t *p, uint64_t n_words)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride)
        p[i] = 0;
}

// Popcount histogram of the blocks: eight lanes read one block's eight
// words (coalesced), sum their popcounts with lane swizzles inside the
// group, and bump a workgroup histogram in LDS; non-empty bins are added to
// the global histogram at the end. The grid stride is a multiple of 8
// words, so every group of eight lanes stays on one block.
__global__ __launch_bounds__(256) void load_histogram_kernel(const uint64_t *__restrict__ words, uint64_t n_words,
                                                            unsigned long long *__restrict__ hist)
{
    __shared__ uint32_t sh[513];
    for (uint32_t i = threadIdx.x; i < 513; i += blockDim.x)
        sh[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_words; w += stride) {
        uint32_t pc = (uint32_t)__popcll(words[w]);
        pc += __shfl_xor(pc, 1);
        pc += __shfl_xor(pc, 2);
        pc += __shfl_xor(pc, 4);
        if ((threadIdx.x & 7) == 0)
            atomicAdd(&sh[pc], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 513; i += blockDim.x)
        if (sh[i])
            atomicAdd(&hist[i], (unsigned long long)sh[i]);
}

// ------------------------------------------------------------ launchers

KParams make_kparams(const bbfc_filter &f)
{
    KParams p{};
    p.words = f.d_words;
    p.rank = f.d_rank;
    p.blk = f.blk;
    p.sub = f.sub;
    p.sub_mult = f.sub_mult;
    p.k = f.k;
    p.c = f.c;
    p.distinct = f.bit_selection == BBFC_BITS_DISTINCT ? 1u : 0u;
    for (uint32_t i = 0; i < f.c; ++i)
        p.block_mult[i] = f.block_mult[i];
    for (uint32_t i = 0; i < f.k; ++i)
        p.bit_mult[i] = f.bit_mult[i];
    return p;
}

uint64_t insert_inflight(const bbfc_filter &f)
{
    uint64_t lim = f.max_inflight;
    if (lim == 0) {
        // One candidate: the filter is the OR of every key's mask in any
        // order, so nothing is gained by holding keys back.
        if (f.c == 1)
            return UINT64_MAX >> 8;
        // A decision can miss bits that keys still in flight are about to
        // set in the candidates it weighs; the drift of the false-positive
        // rate grows with keys in flight per block and with the number of
        // other candidates weighed, c - 1.
        lim = f.M / (8 * (uint64_t)(f.c - 1));
    }
    return lim < (uint64_t)kTile ? (uint64_t)kTile : lim;
}

// Bounds up to this many keys in flight take the tiles of 8 keys: there the
// wide tiles would leave most of the GPU idle and each wavefront's own
// latency sets the rate.
constexpr uint64_t kNarrowMaxInflight = 1u << 16;
// Workgroups of tiles of 8 keys per CU at most (128 keys): more resident
// workgroups lowered the rate (on 2^18- and 2^25-block filters).
constexpr int kNarrowWgsPerCU = 4;

uint32_t insert_tile_keys(const bbfc_filter &f)
{
    if (f.insert_tile != 0)
        return f.insert_tile == 2 ? (uint32_t)kNarrowKeys : (uint32_t)kTile;
    return insert_inflight(f) <= kNarrowMaxInflight ? (uint32_t)kNarrowKeys : (uint32_t)kTile;
}

size_t rank_lds_bytes(uint32_t c, uint32_t k)
{
    return c > 1 ? (size_t)(k + 1) * kRankStride * sizeof(uint16_t) : 0;
}

namespace {

template <int V>
using IC = std::integral_constant<int, V>;

// Calls fn(IC<LPK>, IC<T>) for the configured lanes per key and tiles per wave.
template <typename Fn>
hipError_t with_shape(int lpk, int tpw, Fn &&fn)
{
    if (lpk == 4)
        return tpw == 2 ? fn(IC<4>{}, IC<2>{}) : fn(IC<4>{}, IC<1>{});
    return tpw == 2 ? fn(IC<8>{}, IC<2>{}) : fn(IC<8>{}, IC<1>{});
}

// Workgroups to launch: resident capacity (optionally capped per CU),
// at most what the work needs, at least one.
template <typename K>
uint64_t grid_for(K kernel, size_t dyn_lds, int num_cus, int wgs_per_cu, uint64_t need)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWGSize, dyn_lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (wgs_per_cu > 0 && wgs_per_cu < per_cu)
        per_cu = wgs_per_cu;
    uint64_t wgs = (uint64_t)per_cu * (uint64_t)(num_cus > 0 ? num_cus : 1);
    if (need < wgs)
        wgs = need;
    return wgs < 1 ? 1 : wgs;
}

template <int C, int LPK, int T, typename Src, bool REC = false>
hipError_t insert_launch(const bbfc_filter &f, const Src &keys, uint64_t n, hipStream_t s, uint8_t *rec = nullptr,
                         InsertGeom *geom = nullptr)
{
    const uint64_t n_units = (n + (uint64_t)T * kTile - 1) / ((uint64_t)T * kTile);
    const size_t lds = rank_lds_bytes(f.c, f.k);
    // keys in flight = working wavefronts * T * 64, bounded by the filter's cap
    uint64_t cap_waves = insert_inflight(f) / ((uint64_t)T * kTile);
    if (cap_waves < 1)
        cap_waves = 1;
    if (cap_waves > n_units)
        cap_waves = n_units;
    const uint64_t need = (cap_waves + kWavesPerWG - 1) / kWavesPerWG;
    if constexpr (REC) {
        const uint64_t wgs = grid_for(insert_recorded_kernel<C, LPK, T, Src>, lds, f.num_cus,
                                      f.shape[BBFC_OP_INSERT].wgs_per_cu, need);
        const uint64_t n_waves = std::min<uint64_t>(wgs * kWavesPerWG, cap_waves);
        hipLaunchKernelGGL((insert_recorded_kernel<C, LPK, T, Src>), dim3((uint32_t)wgs), dim3(kWGSize), lds, s,
                           make_kparams(f), keys, n, n_units, n_waves, rec);
    } else {
        const uint64_t wgs =
            grid_for(insert_kernel<C, LPK, T, Src>, lds, f.num_cus, f.shape[BBFC_OP_INSERT].wgs_per_cu, need);
        const uint64_t n_waves = std::min<uint64_t>(wgs * kWavesPerWG, cap_waves);
        if (geom != nullptr) {
            *geom = InsertGeom{(uint32_t)kTile, (uint32_t)T, n_waves, wgs};
            return hipSuccess;
        }
        hipLaunchKernelGGL((insert_kernel<C, LPK, T, Src>), dim3((uint32_t)wgs), dim3(kWGSize), lds, s,
                           make_kparams(f), keys, n, n_units, n_waves);
    }
    return hipGetLastError();
}

template <int C, typename Src, bool REC = false>
hipError_t insert_narrow_launch(const bbfc_filter &f, const Src &keys, uint64_t n, hipStream_t s, uint8_t *rec,
                                InsertGeom *geom = nullptr)
{
    const uint64_t n_units = (n + kNarrowKeys - 1) / kNarrowKeys;
    uint64_t cap_waves = insert_inflight(f) / kNarrowKeys;
    if (cap_waves < 1)
        cap_waves = 1;
    if (cap_waves > n_units)
        cap_waves = n_units;
    const uint64_t need = (cap_waves + kWavesPerWG - 1) / kWavesPerWG;
    const size_t lds = rank_lds_bytes(f.c, f.k);
    const uint64_t wgs = grid_for(insert_narrow_kernel<C, Src, REC>, lds, f.num_cus, kNarrowWgsPerCU, need);
    const uint64_t n_waves = std::min<uint64_t>(wgs * kWavesPerWG, cap_waves);
    if (geom != nullptr) {
        *geom = InsertGeom{(uint32_t)kNarrowKeys, 1, n_waves, wgs};
        return hipSuccess;
    }
    hipLaunchKernelGGL((insert_narrow_kernel<C, Src, REC>), dim3((uint32_t)wgs), dim3(kWGSize), lds, s,
                       make_kparams(f), keys, n, n_units, n_waves, rec);
    return hipGetLastError();
}

template <int C, int LPK, int T, bool EARLY, typename Src>
hipError_t query_launch(const bbfc_filter &f, const Src &keys, uint64_t n, uint64_t *out, hipStream_t s)
{
    const uint64_t n_units = (n + (uint64_t)T * kTile - 1) / ((uint64_t)T * kTile);
    const uint64_t need = (n_units + kWavesPerWG - 1) / kWavesPerWG;
    const uint64_t wgs =
        grid_for(query_kernel<C, LPK, T, EARLY, Src>, 0, f.num_cus, f.shape[BBFC_OP_QUERY].wgs_per_cu, need);
    hipLaunchKernelGGL((query_kernel<C, LPK, T, EARLY, Src>), dim3((uint32_t)wgs), dim3(kWGSize), 0, s, make_kparams(f),
                       keys, n, out, n_units);
    return hipGetLastError();
}

template <int C, int LPK, int T, bool EARLY>
hipError_t query_pieces_launch(const bbfc_filter &f, QueryPiece *h, QueryPiece *d, uint32_t n_pieces, hipStream_t s)
{
    uint64_t units = 0;
    for (uint32_t i = 0; i < n_pieces; ++i) {
        h[i].unit_off = units;
        units += (h[i].n + (uint64_t)T * kTile - 1) / ((uint64_t)T * kTile);
    }
    if (units == 0)
        return hipSuccess;
    if (n_pieces > kMaxQueryPieces || units > UINT32_MAX)
        return hipErrorInvalidValue; // the kernel stages the first units in 32-bit LDS words
    hipError_t e = hipMemcpyAsync(d, h, n_pieces * sizeof(QueryPiece), hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return e;
    const uint64_t need = (units + kWavesPerWG - 1) / kWavesPerWG;
    const uint64_t wgs =
        grid_for(query_pieces_kernel<C, LPK, T, EARLY>, 0, f.num_cus, f.shape[BBFC_OP_QUERY].wgs_per_cu, need);
    hipLaunchKernelGGL((query_pieces_kernel<C, LPK, T, EARLY>), dim3((uint32_t)wgs), dim3(kWGSize), 0, s,
                       make_kparams(f), d, n_pieces, units);
    return hipGetLastError();
}

template <int C>
hipError_t query_pieces_c(const bbfc_filter &f, QueryPiece *h, QueryPiece *d, uint32_t n_pieces, hipStream_t s)
{
    const bbfc_launch_shape &sh = f.shape[BBFC_OP_QUERY];
    return with_shape(sh.lanes_per_key, sh.tiles_per_wave, [&](auto L, auto T) {
        if constexpr (C > 1) {
            if (f.query_early_exit)
                return query_pieces_launch<C, decltype(L)::value, decltype(T)::value, true>(f, h, d, n_pieces, s);
        }
        return query_pieces_launch<C, decltype(L)::value, decltype(T)::value, false>(f, h, d, n_pieces, s);
    });
}

// Static LDS of insert_kernel<C, LPK, T>: masks and block indices per wave.
constexpr size_t insert_static_lds(int C, int T)
{
    return (size_t)kWavesPerWG * T * kTile * (kSlotDw * sizeof(uint32_t) + C * sizeof(uint64_t));
}

template <int C, typename Src, bool REC = false>
hipError_t insert_c(const bbfc_filter &f, const Src &keys, uint64_t n, hipStream_t s, uint8_t *rec = nullptr,
                    InsertGeom *geom = nullptr)
{
    if (insert_tile_keys(f) == kNarrowKeys)
        return insert_narrow_launch<C, Src, REC>(f, keys, n, s, rec, geom);
    // two tiles per wave only where their LDS and the rank table fit a workgroup
    int tpw = f.shape[BBFC_OP_INSERT].tiles_per_wave;
    if (tpw == 2 && insert_static_lds(C, 2) + rank_lds_bytes(f.c, f.k) > f.max_lds)
        tpw = 1;
    return with_shape(f.shape[BBFC_OP_INSERT].lanes_per_key, tpw, [&](auto L, auto T) {
        return insert_launch<C, decltype(L)::value, decltype(T)::value, Src, REC>(f, keys, n, s, rec, geom);
    });
}

template <int C, typename Src>
hipError_t query_c(const bbfc_filter &f, const Src &keys, uint64_t n, uint64_t *out, hipStream_t s)
{
    const bbfc_launch_shape &sh = f.shape[BBFC_OP_QUERY];
    return with_shape(sh.lanes_per_key, sh.tiles_per_wave, [&](auto L, auto T) {
        if constexpr (C > 1) {
            if (f.query_early_exit)
                return query_launch<C, decltype(L)::value, decltype(T)::value, true, Src>(f, keys, n, out, s);
        }
        return query_launch<C, decltype(L)::value, decltype(T)::value, false, Src>(f, keys, n, out, s);
    });
}

template <typename Src, bool REC = false>
hipError_t insert_any(const bbfc_filter &f, const Src &keys, uint64_t n, hipStream_t s, uint8_t *rec = nullptr,
                      InsertGeom *geom = nullptr)
{
    switch (f.c) {
    case 1:
        return insert_c<1, Src, REC>(f, keys, n, s, rec, geom);
    case 2:
        return insert_c<2, Src, REC>(f, keys, n, s, rec, geom);
    case 3:
        return insert_c<3, Src, REC>(f, keys, n, s, rec, geom);
    case 4:
        return insert_c<4, Src, REC>(f, keys, n, s, rec, geom);
    default:
        return hipErrorInvalidValue;
    }
}

template <typename Src>
hipError_t query_any(const bbfc_filter &f, const Src &keys, uint64_t n, uint64_t *out, hipStream_t s)
{
    switch (f.c) {
    case 1:
        return query_c<1>(f, keys, n, out, s);
    case 2:
        return query_c<2>(f, keys, n, out, s);
    case 3:
        return query_c<3>(f, keys, n, out, s);
    case 4:
        return query_c<4>(f, keys, n, out, s);
    default:
        return hipErrorInvalidValue;
    }
}

// One thread per key: the canonical k-mers written out.
__global__ void kmer_keys_kernel(KmerKeys src, uint64_t n, uint64_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        out[t] = src.load(t);
}

KmerKeys make_kmer_src(const uint64_t *seq, uint64_t seg_len, uint32_t q)
{
    KmerKeys src{};
    src.seq = seq;
    src.seg_len = seg_len;
    src.per_seg = seg_len >= q ? seg_len - q + 1 : 0;
    const FastMod fm = make_fastmod(src.per_seg ? src.per_seg : 1);
    src.fm_magic = fm.magic;
    src.fm_sh1 = fm.sh1;
    src.fm_sh2 = fm.sh2;
    src.q = q;
    return src;
}

} // namespace

hipError_t launch_insert(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    return insert_any(f, ArrayKeys{keys}, n, s);
}

hipError_t insert_geometry(const bbfc_filter &f, uint64_t n, InsertGeom *geom)
{
    return insert_any(f, ArrayKeys{nullptr}, n, nullptr, nullptr, geom);
}

hipError_t launch_insert_recorded(const bbfc_filter &f, const uint64_t *keys, uint64_t n, uint8_t *decisions,
                                  hipStream_t s)
{
    return insert_any<ArrayKeys, true>(f, ArrayKeys{keys}, n, s, decisions);
}

hipError_t launch_insert_kmers(const bbfc_filter &f, const uint64_t *seq, uint64_t n_segments, uint64_t seg_len, uint32_t q, hipStream_t s)
{
    const KmerKeys src = make_kmer_src(seq, seg_len, q);
    return insert_any(f, src, n_segments * src.per_seg, s);
}

hipError_t launch_query_kmers(const bbfc_filter &f, const uint64_t *seq, uint64_t n_segments, uint64_t seg_len, uint32_t q, uint64_t *out, hipStream_t s)
{
    const KmerKeys src = make_kmer_src(seq, seg_len, q);
    return query_any(f, src, n_segments * src.per_seg, out, s);
}

hipError_t launch_kmer_keys(const uint64_t *seq, uint64_t n_segments, uint64_t seg_len, uint32_t q, uint64_t *out,
                            hipStream_t s)
{
    const KmerKeys src = make_kmer_src(seq, seg_len, q);
    const uint64_t n = n_segments * src.per_seg;
    if (n == 0)
        return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(kmer_keys_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, src, n, out);
    return hipGetLastError();
}

hipError_t launch_query(const bbfc_filter &f, const uint64_t *keys, uint64_t n, uint64_t *out, hipStream_t s)
{
    return query_any(f, ArrayKeys{keys}, n, out, s);
}

hipError_t launch_query_pieces(const bbfc_filter &f, QueryPiece *h_pieces, QueryPiece *d_pieces, uint32_t n_pieces,
                               hipStream_t s)
{
    switch (f.c) {
    case 1:
        return query_pieces_c<1>(f, h_pieces, d_pieces, n_pieces, s);
    case 2:
        return query_pieces_c<2>(f, h_pieces, d_pieces, n_pieces, s);
    case 3:
        return query_pieces_c<3>(f, h_pieces, d_pieces, n_pieces, s);
    case 4:
        return query_pieces_c<4>(f, h_pieces, d_pieces, n_pieces, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_load_histogram(const bbfc_filter &f, uint64_t *hist, hipStream_t s)
{
    hipError_t e = launch_fill_zero(hist, 513, s);
    if (e != hipSuccess)
        return e;
    const uint64_t n_words = f.M * 8; // a multiple of 8: groups of 8 lanes never straddle the end
    uint64_t blocks = (n_words + 255) / 256;
    const uint64_t cap = (uint64_t)(f.num_cus > 0 ? f.num_cus : 256) * 8;
    if (blocks > cap)
        blocks = cap;
    hipLaunchKernelGGL(load_histogram_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, f.d_words, n_words,
                       reinterpret_cast<unsigned long long *>(hist));
    return hipGetLastError();
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
