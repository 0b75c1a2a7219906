// Batches of filters built or queried in one persistent launch, their
// hipGraph capture, and the launch-shape autotuner.
//
// A plan lists the filters, the number of keys each receives per call, and
// the layout of the concatenated key and answer arrays. Its device copy is a
// table of per-filter descriptors (the same KParams the single-filter
// kernels receive as arguments, plus offsets).
//
// Query: the answer-producing work is cut into units of T tiles of 64 keys,
// numbered filter after filter; resident wavefronts take units in strides
// and find each unit's filter with a cursor that only moves forward.
//
// Insert: racing inserts must keep, per filter, no more keys in flight than
// that filter's cap (the single-filter launcher bounds the grid for the same
// reason). Each filter's units are split into `slots`, at most cap/(64 T) of
// them; a slot is a strided sequence of units processed in order by one
// wavefront. Wavefronts pull slots from an atomic counter, longest slots
// first, until none are left, so a filter never has more slots running than
// it has slots.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include <hip/hip_runtime.h>

#include "bbfc_common.hpp"
#include "bbfc_internal.hpp"
#include "bbfc_tile.hpp"

namespace bbfc {

namespace {

constexpr int kWavesPerWG = 4;
constexpr int kWGSize = kWave * kWavesPerWG;

struct BatchFilter {
    KParams p;
    uint64_t key_off;  // first key of the filter in the concatenated keys
    uint64_t n;        // keys of the filter per call
    uint64_t out_off;  // first answer word of the filter
    uint64_t unit_off; // first query unit of the filter (depends on T)
};

struct BatchSlot {
    uint32_t filter;
    uint32_t first_unit;
    uint32_t stride;
    uint32_t units; // units of the filter
};

__device__ inline uint32_t wave_index()
{
    return (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// The first active lane's 64-bit value, as a wave-uniform value.
__device__ inline uint64_t first_lane_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Work counters: one queue per XCD, each counter on its own 128-byte line.
// The batch insert uses queue 0's counter for its slots.
constexpr int kQueues = 8;
constexpr int kQueueStride = 16; // 64-bit words between counters
constexpr int kCounterWords = kQueues * kQueueStride;

// Two schedules, chosen per launch: grab == 0 strides units statically over
// the resident wavefronts; grab > 0 hands out units in increasing order,
// `grab` at a time, which keeps the units in flight in one moving window
// (fewer filters read at once, better cache reuse). The blocks of `grab`
// units are dealt to kQueues queues in turn (block b to queue b % kQueues),
// each with its own counter, so that grabs contend on eight addresses rather
// than one: workgroup w draws from queue w % kQueues first (the dispatcher
// places consecutive workgroups on consecutive XCDs), then takes what is
// left in the other queues, so every unit is served wherever the workgroups
// run.
template <int C, int LPK, int T, bool EARLY>
__global__ __launch_bounds__(kWGSize) void batch_query_kernel(const BatchFilter *__restrict__ filt, uint32_t n_filters,
                                                              uint64_t total_units, uint32_t grab,
                                                              unsigned long long *counter,
                                                              const uint64_t *__restrict__ keys,
                                                              uint64_t *__restrict__ out)
{
    __shared__ uint32_t s_mask[kWavesPerWG][T * kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][T * kTile * C];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = wave_index();
    uint32_t f = 0;
    auto unit = [&](uint64_t u) __attribute__((always_inline)) {
        if (filt[f].unit_off > u) // a queue taken over from another XCD starts lower
            f = 0;
        while (f + 1 < n_filters && filt[f + 1].unit_off <= u)
            ++f;
        const BatchFilter &bf = filt[f];
        const uint64_t lu = u - bf.unit_off;
        query_tiles<C, LPK, T, EARLY>(bf.p, ArrayKeys{keys + bf.key_off}, bf.n, lu * T * kTile,
                                      out + bf.out_off + lu * T, lane, s_mask[wv], s_blk[wv]);
    };
    if (grab == 0) {
        const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerWG;
        for (uint64_t u = (uint64_t)blockIdx.x * kWavesPerWG + wv; u < total_units; u += n_waves)
            unit(u);
        return;
    }
    const uint64_t n_blocks = (total_units + grab - 1) / grab;
    const uint32_t q0 = blockIdx.x % kQueues;
    for (uint32_t qi = 0; qi < kQueues; ++qi) {
        const uint32_t q = (q0 + qi) % kQueues;
        for (;;) {
            unsigned long long i = 0;
            if (lane == 0)
                i = atomicAdd(counter + q * kQueueStride, 1ull);
            const uint64_t b = first_lane_u64(i) * kQueues + q;
            if (b >= n_blocks)
                break;
            const uint64_t first = b * grab;
            const uint64_t last = first + grab < total_units ? first + grab : total_units;
            for (uint64_t u = first; u < last; ++u)
                unit(u);
        }
    }
}

template <int C, int LPK, int T>
__global__ __launch_bounds__(kWGSize) void batch_insert_kernel(const BatchFilter *__restrict__ filt,
                                                               const BatchSlot *__restrict__ slots, uint32_t n_slots,
                                                               unsigned long long *counter,
                                                               const uint64_t *__restrict__ keys)
{
    __shared__ uint32_t s_mask[kWavesPerWG][T * kTile * kSlotDw];
    __shared__ uint64_t s_blk[kWavesPerWG][T * kTile * C];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = wave_index();
    for (;;) {
        unsigned long long s = 0;
        if (lane == 0)
            s = atomicAdd(counter, 1ull);
        s = first_lane_u64(s);
        if (s >= n_slots)
            break;
        const BatchSlot sl = slots[s];
        const BatchFilter &bf = filt[sl.filter];
        for (uint64_t lu = sl.first_unit; lu < sl.units; lu += sl.stride)
            insert_tiles<C, LPK, T>(bf.p, bf.p.rank, ArrayKeys{keys + bf.key_off}, bf.n, lu * T * kTile, lane,
                                    s_mask[wv], s_blk[wv]);
    }
}

// Zeroes the persistent kernels' work counters (a kernel rather than a
// memset, so that graphs replay it correctly).
__global__ void reset_counter_kernel(unsigned long long *counter)
{
    for (int i = threadIdx.x; i < kCounterWords; i += blockDim.x)
        counter[i] = 0;
}

template <int V>
using IC = std::integral_constant<int, V>;

template <typename Fn>
hipError_t with_shape(int lpk, int tpw, Fn &&fn)
{
    if (lpk == 4)
        return tpw == 2 ? fn(IC<4>{}, IC<2>{}) : fn(IC<4>{}, IC<1>{});
    return tpw == 2 ? fn(IC<8>{}, IC<2>{}) : fn(IC<8>{}, IC<1>{});
}

template <typename Fn>
hipError_t with_choices(uint32_t c, Fn &&fn)
{
    switch (c) {
    case 1:
        return fn(IC<1>{});
    case 2:
        return fn(IC<2>{});
    case 3:
        return fn(IC<3>{});
    case 4:
        return fn(IC<4>{});
    default:
        return hipErrorInvalidValue;
    }
}

template <typename K>
uint64_t resident_wgs(K kernel, int num_cus, int wgs_per_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWGSize, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (wgs_per_cu > 0 && wgs_per_cu < per_cu)
        per_cu = wgs_per_cu;
    return (uint64_t)per_cu * (uint64_t)(num_cus > 0 ? num_cus : 1);
}

bool same_shape(const bbfc_launch_shape &a, const bbfc_launch_shape &b)
{
    return a.lanes_per_key == b.lanes_per_key && a.tiles_per_wave == b.tiles_per_wave &&
           a.wgs_per_cu == b.wgs_per_cu && a.units_per_grab == b.units_per_grab;
}

bool valid_shape(const bbfc_launch_shape &s)
{
    return (s.lanes_per_key == 4 || s.lanes_per_key == 8) && (s.tiles_per_wave == 1 || s.tiles_per_wave == 2) &&
           s.wgs_per_cu >= 0 && s.wgs_per_cu <= 64 && s.units_per_grab >= 0 && s.units_per_grab <= 4096;
}

} // namespace
} // namespace bbfc

namespace bbfc {
namespace {
// Device tables one launch of a plan reads.
struct Tables {
    BatchFilter *d_filt = nullptr;
    BatchSlot *d_slots = nullptr;
    unsigned long long *d_counter = nullptr;
    uint32_t n_filters = 0;
    uint32_t n_slots = 0;
    uint64_t total_units = 0;
    size_t slot_bytes = 0;
};
} // namespace
} // namespace bbfc

struct bbfc_batch {
    std::vector<bbfc_handle> filters;
    std::vector<uint64_t> n_keys;
    uint32_t c = 0;
    int device = 0;
    int num_cus = 0;
    uint64_t total_keys = 0;
    uint64_t total_words = 0;
    // [BBFC_OP_INSERT], [BBFC_OP_QUERY]; queries take units in order, 8 per
    // grab, so that few filters are read at once
    bbfc_launch_shape shape[2] = {{8, 1, 0, 1, 0.0f}, {8, 1, 0, 8, 0.0f}};
    // device tables, rebuilt when a shape changes (graphs keep their own copies)
    bbfc::Tables t;
    int tables_tpw_query = 0;
    int tables_tpw_insert = 0;
    std::vector<bbfc::BatchFilter> h_filt;
};

struct bbfc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    bbfc::Tables tables[2]; // copies of the captured plans' tables, owned by the graph
};

namespace bbfc {
namespace {

uint64_t units_of(uint64_t n, int tpw)
{
    const uint64_t tiles = (n + kTile - 1) / kTile;
    return (tiles + (uint64_t)tpw - 1) / (uint64_t)tpw;
}

void free_tables(Tables &t, bool with_counter)
{
    if (t.d_filt)
        (void)hipFree(t.d_filt);
    if (t.d_slots)
        (void)hipFree(t.d_slots);
    t.d_filt = nullptr;
    t.d_slots = nullptr;
    if (with_counter && t.d_counter) {
        (void)hipFree(t.d_counter);
        t.d_counter = nullptr;
    }
}

// A private copy of a plan's tables (and its own work counter).
hipError_t copy_tables(const Tables &src, Tables &dst)
{
    dst = src;
    dst.d_filt = nullptr;
    dst.d_slots = nullptr;
    dst.d_counter = nullptr;
    hipError_t e = hipMalloc(&dst.d_filt, src.n_filters * sizeof(BatchFilter));
    if (e == hipSuccess)
        e = hipMalloc(&dst.d_slots, src.slot_bytes);
    if (e == hipSuccess)
        e = hipMalloc(&dst.d_counter, kCounterWords * sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipMemcpy(dst.d_filt, src.d_filt, src.n_filters * sizeof(BatchFilter), hipMemcpyDeviceToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(dst.d_slots, src.d_slots, src.slot_bytes, hipMemcpyDeviceToDevice);
    if (e != hipSuccess)
        free_tables(dst, true);
    return e;
}

// (Re)builds the descriptor table for the query unit size and the slot
// table for the insert unit size, and uploads both.
bbfc_status build_tables(bbfc_batch &b)
{
    const int tq = b.shape[BBFC_OP_QUERY].tiles_per_wave;
    const int ti = b.shape[BBFC_OP_INSERT].tiles_per_wave;
    if (b.t.d_filt && tq == b.tables_tpw_query && ti == b.tables_tpw_insert)
        return BBFC_OK;
    const uint32_t nf = (uint32_t)b.filters.size();
    b.h_filt.assign(nf, BatchFilter{});
    uint64_t koff = 0, woff = 0, uoff = 0;
    std::vector<BatchSlot> slots;
    for (uint32_t f = 0; f < nf; ++f) {
        BatchFilter &d = b.h_filt[f];
        d.p = make_kparams(*b.filters[f]);
        d.key_off = koff;
        d.n = b.n_keys[f];
        d.out_off = woff;
        d.unit_off = uoff;
        koff += b.n_keys[f];
        woff += (b.n_keys[f] + 63) / 64;
        uoff += units_of(b.n_keys[f], tq);
        const uint64_t iu = units_of(b.n_keys[f], ti);
        if (iu == 0)
            continue;
        if (iu > UINT32_MAX)
            return fail(BBFC_EINVAL, "filter %u has too many keys for a batch", f);
        uint64_t ns = insert_inflight(*b.filters[f]) / ((uint64_t)ti * kTile);
        ns = std::max<uint64_t>(1, std::min<uint64_t>(ns, iu));
        for (uint64_t s = 0; s < ns; ++s)
            slots.push_back(BatchSlot{f, (uint32_t)s, (uint32_t)ns, (uint32_t)iu});
    }
    // longest slots first
    std::stable_sort(slots.begin(), slots.end(), [](const BatchSlot &x, const BatchSlot &y) {
        const uint64_t lx = (x.units - x.first_unit + x.stride - 1) / x.stride;
        const uint64_t ly = (y.units - y.first_unit + y.stride - 1) / y.stride;
        return lx > ly;
    });
    if (slots.size() > UINT32_MAX)
        return fail(BBFC_EINVAL, "too many insert slots");
    DeviceGuard guard(b.device);
    free_tables(b.t, false);
    hipError_t e = hipMalloc(&b.t.d_filt, nf * sizeof(BatchFilter));
    b.t.slot_bytes = std::max<size_t>(1, slots.size()) * sizeof(BatchSlot);
    if (e == hipSuccess)
        e = hipMalloc(&b.t.d_slots, b.t.slot_bytes);
    if (e == hipSuccess)
        e = hipMemcpy(b.t.d_filt, b.h_filt.data(), nf * sizeof(BatchFilter), hipMemcpyHostToDevice);
    if (e == hipSuccess && !slots.empty())
        e = hipMemcpy(b.t.d_slots, slots.data(), slots.size() * sizeof(BatchSlot), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_tables(b.t, false);
        b.tables_tpw_query = 0;
        return hip_fail(e, "uploading batch tables");
    }
    b.t.n_filters = nf;
    b.t.n_slots = (uint32_t)slots.size();
    b.t.total_units = uoff;
    b.tables_tpw_query = tq;
    b.tables_tpw_insert = ti;
    return BBFC_OK;
}

hipError_t launch_batch_query(const Tables &t, uint32_t c, int num_cus, const bbfc_launch_shape &sh,
                              const uint64_t *keys, uint64_t *out, hipStream_t s)
{
    if (t.total_units == 0)
        return hipSuccess;
    const uint32_t grab = (uint32_t)sh.units_per_grab;
    if (grab > 0) {
        hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, t.d_counter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return with_choices(c, [&](auto Cc) {
        constexpr int C = decltype(Cc)::value;
        return with_shape(sh.lanes_per_key, sh.tiles_per_wave, [&](auto L, auto Tt) {
            constexpr int LPK = decltype(L)::value;
            constexpr int T = decltype(Tt)::value;
            constexpr bool EARLY = C > 1;
            auto kern = batch_query_kernel<C, LPK, T, EARLY>;
            uint64_t wgs = resident_wgs(kern, num_cus, sh.wgs_per_cu);
            const uint64_t chunks = (t.total_units + (grab ? grab : 1) - 1) / (grab ? grab : 1);
            const uint64_t need = (chunks + kWavesPerWG - 1) / kWavesPerWG;
            wgs = std::max<uint64_t>(1, std::min(wgs, need));
            hipLaunchKernelGGL(kern, dim3((uint32_t)wgs), dim3(kWGSize), 0, s, t.d_filt, t.n_filters, t.total_units,
                               grab, t.d_counter, keys, out);
            return hipGetLastError();
        });
    });
}

hipError_t launch_batch_insert(const Tables &t, uint32_t c, int num_cus, const bbfc_launch_shape &sh,
                               const uint64_t *keys, hipStream_t s)
{
    if (t.n_slots == 0)
        return hipSuccess;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, t.d_counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return with_choices(c, [&](auto Cc) {
        constexpr int C = decltype(Cc)::value;
        return with_shape(sh.lanes_per_key, sh.tiles_per_wave, [&](auto L, auto Tt) {
            constexpr int LPK = decltype(L)::value;
            constexpr int T = decltype(Tt)::value;
            auto kern = batch_insert_kernel<C, LPK, T>;
            uint64_t wgs = resident_wgs(kern, num_cus, sh.wgs_per_cu);
            const uint64_t need = (t.n_slots + kWavesPerWG - 1) / kWavesPerWG;
            wgs = std::max<uint64_t>(1, std::min(wgs, need));
            hipLaunchKernelGGL(kern, dim3((uint32_t)wgs), dim3(kWGSize), 0, s, t.d_filt, t.d_slots, t.n_slots,
                               t.d_counter, keys);
            return hipGetLastError();
        });
    });
}

hipError_t plan_insert(const bbfc_batch &b, const uint64_t *keys, hipStream_t s)
{
    return launch_batch_insert(b.t, b.c, b.num_cus, b.shape[BBFC_OP_INSERT], keys, s);
}

hipError_t plan_query(const bbfc_batch &b, const uint64_t *keys, uint64_t *out, hipStream_t s)
{
    return launch_batch_query(b.t, b.c, b.num_cus, b.shape[BBFC_OP_QUERY], keys, out, s);
}

bbfc_status check_op(int32_t op)
{
    if (op != BBFC_OP_INSERT && op != BBFC_OP_QUERY)
        return fail(BBFC_EINVAL, "op must be BBFC_OP_INSERT or BBFC_OP_QUERY");
    return BBFC_OK;
}

} // namespace
} // namespace bbfc

using bbfc::fail;
using bbfc::hip_fail;

extern "C" {

bbfc_status bbfc_batch_create(const bbfc_handle *filters, const uint64_t *n_keys, uint32_t n_filters,
                              bbfc_batch_handle *out)
{
    if (filters == nullptr || n_keys == nullptr || out == nullptr || n_filters == 0)
        return fail(BBFC_EINVAL, "batch needs filters, key counts, an output handle and n_filters > 0");
    for (uint32_t f = 0; f < n_filters; ++f) {
        if (filters[f] == nullptr)
            return fail(BBFC_EINVAL, "filter %u is null", f);
        if (filters[f]->c != filters[0]->c)
            return fail(BBFC_EINVAL, "all filters of a batch must have the same number of choices");
        if (filters[f]->device != filters[0]->device)
            return fail(BBFC_EINVAL, "all filters of a batch must live on one device");
    }
    auto *b = new bbfc_batch();
    b->filters.assign(filters, filters + n_filters);
    b->n_keys.assign(n_keys, n_keys + n_filters);
    b->c = filters[0]->c;
    b->device = filters[0]->device;
    b->num_cus = filters[0]->num_cus;
    for (uint32_t f = 0; f < n_filters; ++f) {
        b->total_keys += n_keys[f];
        b->total_words += (n_keys[f] + 63) / 64;
    }
    bbfc::DeviceGuard guard(b->device);
    hipError_t e = hipMalloc(&b->t.d_counter, bbfc::kCounterWords * sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "allocating the batch counter");
    }
    bbfc_status st = bbfc::build_tables(*b);
    if (st != BBFC_OK) {
        bbfc_batch_destroy(b);
        return st;
    }
    *out = b;
    return BBFC_OK;
}

bbfc_status bbfc_batch_destroy(bbfc_batch_handle b)
{
    if (b == nullptr)
        return fail(BBFC_EINVAL, "null batch");
    bbfc::DeviceGuard guard(b->device);
    hipError_t e = hipDeviceSynchronize();
    bbfc::free_tables(b->t, true);
    delete b;
    return e == hipSuccess ? BBFC_OK : hip_fail(e, "synchronising before batch destroy");
}

bbfc_status bbfc_batch_layout(bbfc_batch_handle b, uint64_t *total_keys, uint64_t *total_out_words)
{
    if (b == nullptr)
        return fail(BBFC_EINVAL, "null batch");
    if (total_keys)
        *total_keys = b->total_keys;
    if (total_out_words)
        *total_out_words = b->total_words;
    return BBFC_OK;
}

bbfc_status bbfc_batch_insert(bbfc_batch_handle b, const uint64_t *d_keys, hipStream_t stream)
{
    if (b == nullptr)
        return fail(BBFC_EINVAL, "null batch");
    if (b->total_keys == 0)
        return BBFC_OK;
    if (d_keys == nullptr)
        return fail(BBFC_EINVAL, "null keys");
    bbfc::DeviceGuard guard(b->device);
    bbfc_status st = bbfc::build_tables(*b);
    if (st != BBFC_OK)
        return st;
    hipError_t e = bbfc::plan_insert(*b, d_keys, stream);
    return e == hipSuccess ? BBFC_OK : hip_fail(e, "launching batch insert");
}

bbfc_status bbfc_batch_query(bbfc_batch_handle b, const uint64_t *d_keys, uint64_t *d_out_bits, hipStream_t stream)
{
    if (b == nullptr)
        return fail(BBFC_EINVAL, "null batch");
    if (b->total_keys == 0)
        return BBFC_OK;
    if (d_keys == nullptr || d_out_bits == nullptr)
        return fail(BBFC_EINVAL, "null keys or output");
    const uintptr_t k0 = (uintptr_t)d_keys, k1 = k0 + b->total_keys * 8;
    const uintptr_t o0 = (uintptr_t)d_out_bits, o1 = o0 + b->total_words * 8;
    if (k0 < o1 && o0 < k1)
        return fail(BBFC_EINVAL, "output overlaps the keys");
    bbfc::DeviceGuard guard(b->device);
    bbfc_status st = bbfc::build_tables(*b);
    if (st != BBFC_OK)
        return st;
    hipError_t e = bbfc::plan_query(*b, d_keys, d_out_bits, stream);
    return e == hipSuccess ? BBFC_OK : hip_fail(e, "launching batch query");
}

bbfc_status bbfc_batch_set_shape(bbfc_batch_handle b, int32_t op, bbfc_launch_shape shape)
{
    if (b == nullptr)
        return fail(BBFC_EINVAL, "null batch");
    bbfc_status st = bbfc::check_op(op);
    if (st != BBFC_OK)
        return st;
    if (!bbfc::valid_shape(shape))
        return fail(BBFC_EINVAL, "shape: lanes_per_key 4|8, tiles_per_wave 1|2, wgs_per_cu 0..64");
    b->shape[op] = shape;
    return bbfc::build_tables(*b);
}

bbfc_status bbfc_batch_get_shape(bbfc_batch_handle b, int32_t op, bbfc_launch_shape *shape)
{
    if (b == nullptr || shape == nullptr)
        return fail(BBFC_EINVAL, "null batch or output");
    bbfc_status st = bbfc::check_op(op);
    if (st != BBFC_OK)
        return st;
    *shape = b->shape[op];
    return BBFC_OK;
}

bbfc_status bbfc_batch_tune(bbfc_batch_handle b, int32_t op, const uint64_t *d_keys, uint64_t *d_out_bits,
                            uint32_t reps, hipStream_t stream, bbfc_launch_shape *best)
{
    if (b == nullptr || d_keys == nullptr || (op == BBFC_OP_QUERY && d_out_bits == nullptr))
        return fail(BBFC_EINVAL, "null batch, keys or output");
    bbfc_status st = bbfc::check_op(op);
    if (st != BBFC_OK)
        return st;
    if (reps == 0)
        reps = 1;
    bbfc::DeviceGuard guard(b->device);
    const bbfc_launch_shape saved = b->shape[op];

    // Insert trials change the filters: snapshot them and restore before
    // every trial and at the end.
    std::vector<uint64_t *> snap;
    hipError_t e = hipSuccess;
    if (op == BBFC_OP_INSERT) {
        for (bbfc_handle f : b->filters) {
            uint64_t *p = nullptr;
            e = hipMalloc(&p, f->M * 64);
            if (e != hipSuccess)
                break;
            snap.push_back(p);
            e = hipMemcpyAsync(p, f->d_words, f->M * 64, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess)
                break;
        }
    }
    auto restore = [&]() -> hipError_t {
        hipError_t r = hipSuccess;
        for (size_t i = 0; i < snap.size() && r == hipSuccess; ++i)
            r = hipMemcpyAsync(b->filters[i]->d_words, snap[i], b->filters[i]->M * 64, hipMemcpyDeviceToDevice,
                               stream);
        return r;
    };
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (e == hipSuccess)
        e = hipEventCreate(&ev0);
    if (e == hipSuccess)
        e = hipEventCreate(&ev1);

    bbfc_launch_shape winner = saved;
    float best_ms = -1.0f;
    // Candidates: lanes per key x tiles per wavefront x occupancy cap, and
    // for queries the schedule (static stride, or ordered grabs of 8 units).
    std::vector<bbfc_launch_shape> cands = {saved}; // the shape in force is tried first
    for (int lpk : {8, 4})
        for (int tpw : {1, 2})
            for (int occ : {0, 2})
                for (int grab : {0, 8}) {
                    if (op == BBFC_OP_INSERT && grab == 8)
                        continue; // inserts always take whole slots, one per grab
                    const bbfc_launch_shape c{lpk, tpw, occ, op == BBFC_OP_INSERT ? 1 : grab, 0.0f};
                    if (!bbfc::same_shape(c, saved))
                        cands.push_back(c);
                }
    for (size_t ci = 0; ci < cands.size() && e == hipSuccess && st == BBFC_OK; ++ci) {
        b->shape[op] = cands[ci];
        st = bbfc::build_tables(*b);
        if (st != BBFC_OK)
            break;
        float total = 0.0f;
        for (uint32_t r = 0; r <= reps && e == hipSuccess; ++r) { // r == 0 warms up
            if (op == BBFC_OP_INSERT)
                e = restore();
            if (e == hipSuccess)
                e = hipEventRecord(ev0, stream);
            if (e == hipSuccess)
                e = op == BBFC_OP_INSERT ? bbfc::plan_insert(*b, d_keys, stream)
                                         : bbfc::plan_query(*b, d_keys, d_out_bits, stream);
            if (e == hipSuccess)
                e = hipEventRecord(ev1, stream);
            if (e == hipSuccess)
                e = hipEventSynchronize(ev1);
            float ms = 0.0f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, ev0, ev1);
            if (r > 0)
                total += ms;
        }
        const float avg = total / (float)reps;
        // the shape in force (tried first) keeps its place unless another is
        // more than 2% faster
        const float margin = (ci > 0 && bbfc::same_shape(winner, saved)) ? 0.98f : 1.0f;
        if (e == hipSuccess && (best_ms < 0.0f || avg < best_ms * margin)) {
            best_ms = avg;
            winner = b->shape[op];
            winner.ms = avg;
        }
    }
    if (e == hipSuccess && op == BBFC_OP_INSERT)
        e = restore();
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    for (uint64_t *p : snap)
        (void)hipFree(p);
    if (ev0)
        (void)hipEventDestroy(ev0);
    if (ev1)
        (void)hipEventDestroy(ev1);
    if (st != BBFC_OK) {
        b->shape[op] = saved;
        (void)bbfc::build_tables(*b);
        return st;
    }
    if (e != hipSuccess) {
        b->shape[op] = saved;
        (void)bbfc::build_tables(*b);
        return hip_fail(e, "autotuning");
    }
    b->shape[op] = winner;
    st = bbfc::build_tables(*b);
    if (st != BBFC_OK)
        return st;
    if (best)
        *best = winner;
    return BBFC_OK;
}

bbfc_status bbfc_graph_create(bbfc_batch_handle insert_plan, const uint64_t *d_insert_keys,
                              bbfc_batch_handle query_plan, const uint64_t *d_query_keys, uint64_t *d_out_bits,
                              bbfc_graph_handle *out)
{
    if (out == nullptr || (insert_plan == nullptr && query_plan == nullptr))
        return fail(BBFC_EINVAL, "graph needs an output handle and at least one plan");
    if (insert_plan && insert_plan->total_keys && d_insert_keys == nullptr)
        return fail(BBFC_EINVAL, "null insert keys");
    if (query_plan && query_plan->total_keys && (d_query_keys == nullptr || d_out_bits == nullptr))
        return fail(BBFC_EINVAL, "null query keys or output");
    if (insert_plan && query_plan && insert_plan->device != query_plan->device)
        return fail(BBFC_EINVAL, "plans of one graph must share a device");
    const int dev = insert_plan ? insert_plan->device : query_plan->device;
    bbfc::DeviceGuard guard(dev);
    bbfc_status st = insert_plan ? bbfc::build_tables(*insert_plan) : BBFC_OK;
    if (st == BBFC_OK && query_plan)
        st = bbfc::build_tables(*query_plan);
    if (st != BBFC_OK)
        return st;

    auto *g = new bbfc_graph();
    g->device = dev;
    hipError_t e = hipSuccess;
    if (insert_plan)
        e = bbfc::copy_tables(insert_plan->t, g->tables[BBFC_OP_INSERT]);
    if (e == hipSuccess && query_plan)
        e = bbfc::copy_tables(query_plan->t, g->tables[BBFC_OP_QUERY]);
    hipStream_t cs = nullptr;
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        if (insert_plan)
            le = bbfc::launch_batch_insert(g->tables[BBFC_OP_INSERT], insert_plan->c, insert_plan->num_cus,
                                           insert_plan->shape[BBFC_OP_INSERT], d_insert_keys, cs);
        if (le == hipSuccess && query_plan)
            le = bbfc::launch_batch_query(g->tables[BBFC_OP_QUERY], query_plan->c, query_plan->num_cus,
                                          query_plan->shape[BBFC_OP_QUERY], d_query_keys, d_out_bits, cs);
        const hipError_t ee = hipStreamEndCapture(cs, &g->graph);
        e = le != hipSuccess ? le : ee;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (cs)
        (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g->graph)
            (void)hipGraphDestroy(g->graph);
        bbfc::free_tables(g->tables[0], true);
        bbfc::free_tables(g->tables[1], true);
        delete g;
        return hip_fail(e, "capturing the batch graph");
    }
    *out = g;
    return BBFC_OK;
}

bbfc_status bbfc_graph_launch(bbfc_graph_handle g, hipStream_t stream)
{
    if (g == nullptr)
        return fail(BBFC_EINVAL, "null graph");
    bbfc::DeviceGuard guard(g->device);
    hipError_t e = hipGraphLaunch(g->exec, stream);
    return e == hipSuccess ? BBFC_OK : hip_fail(e, "launching the graph");
}

bbfc_status bbfc_graph_destroy(bbfc_graph_handle g)
{
    if (g == nullptr)
        return fail(BBFC_EINVAL, "null graph");
    bbfc::DeviceGuard guard(g->device);
    hipError_t e = hipDeviceSynchronize();
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    bbfc::free_tables(g->tables[0], true);
    bbfc::free_tables(g->tables[1], true);
    delete g;
    return e == hipSuccess ? BBFC_OK : hip_fail(e, "synchronising before graph destroy");
}

} // extern "C"
