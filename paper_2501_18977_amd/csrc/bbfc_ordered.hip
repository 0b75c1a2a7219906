// Insert with the sequential semantics on any filter layout (Section 3.2
// applied key by key, in index order).
//
// One workgroup of kOrdThreads threads; each thread holds one key at a time,
// with its 512-bit mask in an LDS slot and its candidate blocks in registers.
// A step
//   1) hashes the keys handed to it by the previous step;
//   2) lets every pending key claim its candidate blocks in a hashed LDS
//      table that keeps the oldest claimer of each entry;
//   3) decides together every pending key that is the oldest claimer of all
//      its entries, reading its candidates from memory and writing the chosen
//      block back, while the next keys, in index order, are loaded for the
//      threads whose key is decided or that held none.
// A key decided in step 3 has no older pending key that shares a candidate
// with it, and two keys decided together share none. A key's candidate
// blocks change only when a key that shares one is inserted; such keys are
// decided before it if older and after it if younger, so every key sees its
// candidates as in the one-at-a-time order. The oldest pending key wins all
// its entries, so each step decides at least one key. A hash collision in the
// table only defers a key to a later step.
//
// Block words are read and written with plain accesses, eight lanes per key
// so that a load reads whole blocks: every thread is in one workgroup, and the
// barrier that ends a step makes its stores visible to the next step's loads
// (workgroup scope; the step also waits for its stores before the barrier).
#include <stdint.h>

#include <mutex>

#include <hip/hip_runtime.h>

#include "bbfc_common.hpp"
#include "bbfc_internal.hpp"
#include "bbfc_tile.hpp"

namespace bbfc {
namespace {

constexpr int kOrdThreads = 1024;
constexpr int kOrdWaves = kOrdThreads / kWave;
constexpr uint32_t kOrdClaims = 8192; // claim table entries, a power of two
constexpr int kOrdSlotDw = 16;        // LDS dwords per key mask

__host__ __device__ constexpr size_t align16(size_t b)
{
    return (b + 15) & ~(size_t)15;
}

// LDS: rank table | key masks | claim table | per-wave counts.
__host__ __device__ constexpr size_t ordered_lds_bytes(size_t rank_bytes)
{
    return align16(rank_bytes) + (size_t)kOrdThreads * kOrdSlotDw * 4 + (size_t)kOrdClaims * 4 + kOrdWaves * 4;
}

// Lane src's 64-bit value.
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t claim_entry(uint64_t blk)
{
    return (uint32_t)blk & (kOrdClaims - 1);
}

template <int C>
__global__ __launch_bounds__(kOrdThreads) void insert_ordered_kernel(KParams p, const uint64_t *__restrict__ keys,
                                                                     uint64_t n, const uint64_t *__restrict__ n_dev,
                                                                     uint32_t rank_bytes)
{
    if (n_dev != nullptr) // the key count is known on the device only
        n = *n_dev;
    extern __shared__ __align__(16) uint8_t lds[];
    uint16_t *s_rank = reinterpret_cast<uint16_t *>(lds);
    uint32_t *smask = reinterpret_cast<uint32_t *>(lds + align16(rank_bytes));
    uint32_t *claim = smask + kOrdThreads * kOrdSlotDw;
    uint32_t *wsum = claim + kOrdClaims;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wv = tid / kWave;
    for (uint32_t i = tid; i < kOrdClaims; i += kOrdThreads)
        claim[i] = 0;
    if constexpr (C > 1) {
        const uint32_t nr = (p.k + 1) * kRankStride;
        for (uint32_t i = tid; i < nr; i += kOrdThreads)
            s_rank[i] = p.rank[i];
    }
    __syncthreads();

    uint32_t *slot = smask + tid * kOrdSlotDw;
    // the first keys go to threads 0, 1, ...; later ones to the threads whose
    // key was decided, in thread order
    uint64_t my = tid;                                             // index of this thread's key
    bool fresh = my < n;                                           // holds a key not hashed yet
    uint64_t xk = fresh ? keys[my] : 0;                            // that key
    uint64_t next = n > (uint64_t)kOrdThreads ? kOrdThreads : n;   // keys handed out (the same in every thread)
    bool pending = false;                                          // holds a key not decided yet
    uint64_t cand[C];
#pragma unroll
    for (int i = 0; i < C; ++i)
        cand[i] = 0;

    for (;;) {
        // 1) hash the keys handed out by the previous step
        if (fresh) {
#pragma unroll
            for (int d = 0; d < kOrdSlotDw; d += 4)
                *reinterpret_cast<uint4 *>(slot + d) = make_uint4(0, 0, 0, 0);
            auto set_bit = [slot](uint32_t f) { atomicOr(slot + (f >> 5), 1u << (f & 31)); };
            if (p.distinct)
                distinct_bits(p.bit_mult, p.k, xk, set_bit);
            else
                random_bits(p.bit_mult, p.k, xk, set_bit);
            const uint64_t first = sub_base(p, xk);
#pragma unroll
            for (int i = 0; i < C; ++i)
                cand[i] = first + block_hash_rt(p, p.block_mult[i], xk);
            pending = true;
            fresh = false;
        }

        // 2) claims: the oldest pending key (largest age) keeps each entry.
        // A key stays pending for at most kOrdThreads steps (each step decides
        // the oldest pending key, and every older key is already held), so
        // ages stay below kOrdThreads * (kOrdThreads + 1) and are distinct.
        const uint32_t age = (uint32_t)(next - my);
        if (pending) {
#pragma unroll
            for (int i = 0; i < C; ++i)
                atomicMax(&claim[claim_entry(cand[i])], age);
        }
        __syncthreads();
        bool ready = pending;
        if (pending) {
#pragma unroll
            for (int i = 0; i < C; ++i)
                ready = ready && claim[claim_entry(cand[i])] == age;
        }
        const bool free_next = !pending || ready;
        const uint64_t fb = __ballot(free_next);
        if (lane == 0)
            wsum[wv] = (uint32_t)__popcll(fb);
        __syncthreads();

        // the next keys, next, next+1, ..., to the threads free after this
        // step; their loads overlap this step's block reads
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kOrdWaves; ++w) {
            const uint32_t c = wsum[w];
            before += (uint32_t)w < wv ? c : 0;
            total += c;
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(fb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fb, 0));
        if (free_next && next + before + below < n) {
            my = next + before + below;
            xk = keys[my];
            fresh = true;
        }
        const uint64_t handed = n - next < total ? n - next : total;
        next += handed;
        // anything left: keys still pending after this step, or keys just handed out
        const bool more = total < (uint32_t)kOrdThreads || handed > 0;
        if (pending) {
#pragma unroll
            for (int i = 0; i < C; ++i)
                claim[claim_entry(cand[i])] = 0;
        }

        // 3) decide the ready keys, eight lanes per key as in the racing
        // insert: round r of a wave takes the wave's keys 8r .. 8r+7, lane
        // group g key 8r+g and block word lane % 8, so each load instruction
        // reads eight whole blocks. The ready keys share no candidate, so all
        // their reads are issued before any write.
        const uint64_t rb = __ballot(ready);
        const uint32_t g = lane / 8;
        const uint32_t w = lane % 8;
        constexpr int RB = C <= 2 ? 8 : 4; // rounds whose reads are in flight together
#pragma unroll
        for (int r0 = 0; r0 < 8; r0 += RB) {
            uint64_t B[RB][C][1];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const uint32_t src = 8 * (r0 + r) + g;
                const bool take = (rb >> src) & 1;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const uint64_t blk = shfl_u64(cand[i], (int)src);
                    B[r][i][0] = take ? p.words[blk * 8 + w] : 0;
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (((rb >> (8 * (r0 + r))) & 0xFF) == 0)
                    continue;
                const uint32_t src = 8 * (r0 + r) + g;
                const bool take = (rb >> src) & 1;
                const uint32_t *ks = smask + (wv * kWave + src) * kOrdSlotDw + 2 * w;
                const uint64_t m[1] = {(uint64_t)ks[0] | ((uint64_t)ks[1] << 32)};
                const JA<C> ja = reduce_ja<C, 8, 1>(B[r], m);
                const int best = decide<C>(ja, s_rank);
                uint64_t blk = shfl_u64(cand[0], (int)src);
#pragma unroll
                for (int i = 1; i < C; ++i) {
                    const uint64_t bi = shfl_u64(cand[i], (int)src);
                    blk = best == i ? bi : blk;
                }
                if (take && best >= 0) {
                    const uint64_t old = pick<C, 1>(B[r], best, 0);
                    if (m[0] & ~old)
                        p.words[blk * 8 + w] = old | m[0];
                }
            }
        }
        if (ready)
            pending = false;
        __builtin_amdgcn_s_waitcnt(0); // this step's stores are done before any thread reads again
        __syncthreads();
        if (!more)
            break;
    }
}

// Checks that the one-workgroup kernel's LDS fits and allows it; done before
// anything is enqueued, so a failure leaves the filter untouched.
template <int C>
hipError_t prepare_ordered_c(const bbfc_filter &f)
{
    const size_t lds = ordered_lds_bytes(rank_lds_bytes(f.c, f.k));
    if (f.max_lds < lds)
        return hipErrorInvalidValue;
    return hipFuncSetAttribute((const void *)insert_ordered_kernel<C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

// Enqueues the one-workgroup kernel (after prepare_ordered_c).
template <int C>
hipError_t enqueue_ordered_c(const bbfc_filter &f, const uint64_t *keys, uint64_t n, const uint64_t *n_dev,
                             hipStream_t s)
{
    const size_t rank = rank_lds_bytes(f.c, f.k);
    hipLaunchKernelGGL((insert_ordered_kernel<C>), dim3(1), dim3(kOrdThreads), ordered_lds_bytes(rank), s,
                       make_kparams(f), keys, n, n_dev, (uint32_t)rank);
    return hipGetLastError();
}

template <int C>
hipError_t launch_ordered_c(const bbfc_filter &f, const uint64_t *keys, uint64_t n, const uint64_t *n_dev,
                            hipStream_t s)
{
    const hipError_t e = prepare_ordered_c<C>(f);
    return e != hipSuccess ? e : enqueue_ordered_c<C>(f, keys, n, n_dev, s);
}

// ------------------------------------------------------------ wide steps
//
// Large inputs go window by window (in index order) through the whole
// device. A window's keys first claim their candidate blocks in a device
// table (hashed by block index) with the value
// (step tag, age): atomicMax keeps the oldest claimer of the current step.
// Then a step decides, across the grid, every pending key of the window that
// still holds all its entries, and the keys that do not claim again for the
// next step; the keys of a step share no candidate and no older pending key
// shares one with them, exactly as in the one-workgroup kernel. A key that
// reads a claim of the next step while checking the current one is only
// deferred. Tags grow with every step of every call, so old entries never
// need clearing. After the plan's steps the one-workgroup kernel inserts the
// window's remaining keys in index order. Kernel boundaries order the steps.

constexpr uint32_t kWideMinKeys = 1u << 16;   // inputs below this stay on one workgroup
constexpr uint32_t kWideMaxWindow = 1u << 18; // the window's scratch is sized for this
constexpr int kWideThreads = 256;

// Window, claim table and steps per filter size. A large filter has few
// conflicts per window: long windows amortise the launches, and a fourth
// step usually leaves no key to the tail.
// A small one has many: shorter windows and more steps leave fewer keys to
// the one-workgroup tail. (Measured on 2^24 keys into 2^25 blocks and 2^22
// keys into 2^17 blocks; every choice gives the same bits.)
struct WidePlan {
    uint32_t window;
    uint64_t claims; // entries, a power of two
    int steps;
};

WidePlan wide_plan(uint64_t n_blocks)
{
    if (n_blocks >= (1ull << 24))
        return {1u << 18, 1ull << 24, 4};
    return {1u << 16, 1ull << 22, 8};
}

// Claim of a key: its step's tag above its age (1 .. window, larger is older).
__device__ __forceinline__ uint64_t claim_value(uint64_t tag, uint32_t age)
{
    return (tag << 24) | age;
}

template <int C>
__device__ __forceinline__ void candidates(const KParams &p, uint64_t x, uint64_t (&cand)[C])
{
    const uint64_t first = sub_base(p, x);
#pragma unroll
    for (int i = 0; i < C; ++i)
        cand[i] = first + block_hash_rt(p, p.block_mult[i], x);
}

template <int C>
__global__ __launch_bounds__(kWideThreads) void wide_claim_kernel(KParams p, const uint64_t *__restrict__ keys,
                                                                  uint32_t w, uint64_t *__restrict__ claims,
                                                                  uint64_t hmask, uint64_t tag,
                                                                  unsigned long long *__restrict__ left)
{
    const uint32_t i = blockIdx.x * kWideThreads + threadIdx.x;
    if (i == 0)
        *left = 0; // the window's last step counts its keys still pending here
    if (i >= w)
        return;
    uint64_t cand[C];
    candidates<C>(p, keys[i], cand);
#pragma unroll
    for (int c = 0; c < C; ++c)
        atomicMax((unsigned long long *)&claims[cand[c] & hmask], (unsigned long long)claim_value(tag, w - i));
}

// One step over a window: thread i holds key i while it is pending.
template <int C>
__global__ __launch_bounds__(kWideThreads) void wide_step_kernel(KParams p, const uint64_t *__restrict__ keys,
                                                                 uint32_t w, uint64_t *__restrict__ claims,
                                                                 uint64_t hmask, uint8_t *__restrict__ pend,
                                                                 uint64_t tag, uint64_t next_tag, int first_step,
                                                                 unsigned long long *__restrict__ left)
{
    extern __shared__ __align__(16) uint8_t lds[];
    uint16_t *s_rank = reinterpret_cast<uint16_t *>(lds);
    const size_t rank_bytes = C > 1 ? align16((size_t)(p.k + 1) * kRankStride * 2) : 0;
    uint32_t *smask = reinterpret_cast<uint32_t *>(lds + rank_bytes);
    if constexpr (C > 1) {
        const uint32_t nr = (p.k + 1) * kRankStride;
        for (uint32_t t = threadIdx.x; t < nr; t += kWideThreads)
            s_rank[t] = p.rank[t];
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t i = blockIdx.x * kWideThreads + threadIdx.x;
    const bool pending = i < w && (first_step || pend[i]);
    const uint64_t x = pending ? keys[i] : 0;
    uint64_t cand[C];
    candidates<C>(p, x, cand);
    const uint64_t mine = claim_value(tag, w - i);
    bool ready = pending;
    if (pending) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            ready = ready && __hip_atomic_load(&claims[cand[c] & hmask], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT) == mine;
    }
    uint32_t *slot = smask + (wv * kWave + lane) * kOrdSlotDw;
    if (ready) {
#pragma unroll
        for (int d = 0; d < kOrdSlotDw; d += 4)
            *reinterpret_cast<uint4 *>(slot + d) = make_uint4(0, 0, 0, 0);
        auto set_bit = [slot](uint32_t f) { atomicOr(slot + (f >> 5), 1u << (f & 31)); };
        if (p.distinct)
            distinct_bits(p.bit_mult, p.k, x, set_bit);
        else
            random_bits(p.bit_mult, p.k, x, set_bit);
    }
    wave_sync();

    // the ready keys of the wavefront, eight lanes per key (as in the racing insert)
    const uint64_t rb = __ballot(ready);
    const uint32_t g = lane / 8;
    const uint32_t wd = lane % 8;
    constexpr int RB = C <= 2 ? 8 : 4;
#pragma unroll
    for (int r0 = 0; r0 < 8; r0 += RB) {
        uint64_t B[RB][C][1];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t src = 8 * (r0 + r) + g;
            const bool take = (rb >> src) & 1;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const uint64_t blk = shfl_u64(cand[c], (int)src);
                B[r][c][0] = take ? p.words[blk * 8 + wd] : 0;
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (((rb >> (8 * (r0 + r))) & 0xFF) == 0)
                continue;
            const uint32_t src = 8 * (r0 + r) + g;
            const bool take = (rb >> src) & 1;
            const uint32_t *ks = smask + (wv * kWave + src) * kOrdSlotDw + 2 * wd;
            const uint64_t m[1] = {(uint64_t)ks[0] | ((uint64_t)ks[1] << 32)};
            const JA<C> ja = reduce_ja<C, 8, 1>(B[r], m);
            const int best = decide<C>(ja, s_rank);
            uint64_t blk = shfl_u64(cand[0], (int)src);
#pragma unroll
            for (int c = 1; c < C; ++c) {
                const uint64_t bc = shfl_u64(cand[c], (int)src);
                blk = best == c ? bc : blk;
            }
            if (take && best >= 0) {
                const uint64_t old = pick<C, 1>(B[r], best, 0);
                if (m[0] & ~old)
                    p.words[blk * 8 + wd] = old | m[0];
            }
        }
    }

    // the others stay pending and claim for the next step (after the last
    // step, they are counted for the tail)
    if (i < w)
        pend[i] = pending && !ready;
    if (next_tag == 0) {
        const uint64_t lb = __ballot(pending && !ready);
        if (lane == 0 && lb != 0)
            atomicAdd(left, (unsigned long long)__popcll(lb));
    }
    if (pending && !ready && next_tag != 0) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            atomicMax((unsigned long long *)&claims[cand[c] & hmask], (unsigned long long)claim_value(next_tag, w - i));
    }
}

// The window's keys still pending, in index order, into tail[0 .. *count).
// Each thread reads 16 flags at a time; nothing is read when the last step
// left no key.
__global__ __launch_bounds__(1024) void wide_tail_kernel(const uint64_t *__restrict__ keys, uint32_t w,
                                                         const uint8_t *__restrict__ pend,
                                                         const unsigned long long *__restrict__ left,
                                                         uint64_t *__restrict__ tail, uint64_t *__restrict__ count)
{
    __shared__ uint32_t wsum[1024 / kWave];
    if (*left == 0) {
        if (threadIdx.x == 0)
            *count = 0;
        return;
    }
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    uint32_t at = 0; // keys written by earlier chunks
    for (uint32_t base = 0; base < w; base += 1024 * 16) {
        const uint32_t i0 = base + threadIdx.x * 16;
        uint32_t flags = 0; // bit j: key i0 + j is pending
        if (i0 + 16 <= w) {
            const uint4 v = *reinterpret_cast<const uint4 *>(pend + i0);
            const uint32_t word[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 16; ++j)
                flags |= ((word[j / 4] >> (8 * (j % 4))) & 0xFF ? 1u : 0u) << j;
        } else {
            for (uint32_t j = 0; i0 + j < w && j < 16; ++j)
                flags |= (pend[i0 + j] ? 1u : 0u) << j;
        }
        // exclusive prefix of the per-thread counts over the workgroup
        const uint32_t mine = (uint32_t)__popc(flags);
        uint32_t x = mine;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, off);
            if (lane >= (uint32_t)off)
                x += y;
        }
        if (lane == kWave - 1)
            wsum[wv] = x;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (uint32_t v = 0; v < 1024 / kWave; ++v) {
            before += v < wv ? wsum[v] : 0;
            total += wsum[v];
        }
        uint32_t o = at + before + x - mine;
        while (flags != 0) {
            const uint32_t j = (uint32_t)__builtin_ctz(flags);
            tail[o++] = keys[i0 + j];
            flags &= flags - 1;
        }
        at += total;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *count = at;
}

// Device memory of the device-wide steps: the claim table, a window's
// pending flags, and its remaining keys followed by their count and the count
// the last step saw. tag holds the last step tag used with this claim table.
struct WideScratch {
    uint64_t *claims;
    uint8_t *pend;
    uint64_t *tail;
    uint64_t *tag;
};

template <int C>
hipError_t run_wide_c(const bbfc_filter &f, const uint64_t *keys, uint64_t n, const WidePlan &plan,
                      const WideScratch &ws, hipStream_t s)
{
    const KParams kp = make_kparams(f);
    const uint64_t hmask = plan.claims - 1;
    const size_t lds = align16(rank_lds_bytes(f.c, f.k)) + (size_t)kWideThreads * kOrdSlotDw * 4;
    uint64_t *count = ws.tail + plan.window;
    unsigned long long *left = reinterpret_cast<unsigned long long *>(ws.tail + plan.window + 1);
    for (uint64_t base = 0; base < n; base += plan.window) {
        const uint32_t w = (uint32_t)(n - base < plan.window ? n - base : plan.window);
        const uint32_t grid = (w + kWideThreads - 1) / kWideThreads;
        const uint64_t *wk = keys + base;
        uint64_t tag = ++*ws.tag;
        hipLaunchKernelGGL((wide_claim_kernel<C>), dim3(grid), dim3(kWideThreads), 0, s, kp, wk, w, ws.claims, hmask,
                           tag, left);
        for (int step = 0; step < plan.steps; ++step) {
            const uint64_t next = step + 1 < plan.steps ? ++*ws.tag : 0;
            hipLaunchKernelGGL((wide_step_kernel<C>), dim3(grid), dim3(kWideThreads), lds, s, kp, wk, w, ws.claims,
                               hmask, ws.pend, tag, next, step == 0 ? 1 : 0, left);
            tag = next;
        }
        hipLaunchKernelGGL(wide_tail_kernel, dim3(1), dim3(1024), 0, s, wk, w, ws.pend, left, ws.tail, count);
        hipError_t e = enqueue_ordered_c<C>(f, ws.tail, 0, count, s);
        if (e != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

template <int C>
hipError_t launch_wide_c(bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    const WidePlan plan = wide_plan(f.M);
    // the tail kernel of every window must fit before the first window runs
    hipError_t e0 = prepare_ordered_c<C>(f);
    if (e0 != hipSuccess)
        return e0;
    if (f.d_ord_claims == nullptr) {
        // scratch of the filter, kept until it is destroyed
        hipError_t e = hipMalloc((void **)&f.d_ord_claims, plan.claims * 8);
        if (e == hipSuccess)
            e = hipMalloc((void **)&f.d_ord_pend, kWideMaxWindow);
        if (e == hipSuccess)
            e = hipMalloc((void **)&f.d_ord_tail, (size_t)kWideMaxWindow * 8 + 16);
        if (e != hipSuccess) {
            // leave nothing half allocated; a later call tries again
            for (void *q : {(void *)f.d_ord_claims, (void *)f.d_ord_pend, (void *)f.d_ord_tail})
                if (q != nullptr)
                    (void)hipFree(q);
            f.d_ord_claims = nullptr;
            f.d_ord_pend = nullptr;
            f.d_ord_tail = nullptr;
            return hipErrorOutOfMemory;
        }
        e = launch_fill_zero(f.d_ord_claims, plan.claims, s);
        if (e != hipSuccess)
            return e;
    }
    // the tail buffer holds the largest window's keys plus two counters
    const WideScratch ws{f.d_ord_claims, f.d_ord_pend, f.d_ord_tail, &f.ord_tag};
    return run_wide_c<C>(f, keys, n, plan, ws, s);
}

template <int C>
hipError_t launch_det_c(bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    if (n < kWideMinKeys)
        return launch_ordered_c<C>(f, keys, n, nullptr, s);
    return launch_wide_c<C>(f, keys, n, s);
}

// ------------------------------------------------- without allocation
//
// The device-wide steps with their scratch in a static device array instead
// of memory the filter allocates: for callers that cannot allocate. Its plan
// is the small-filter one (windows of 2^16 keys, a 2^22-entry claim table) on
// every filter; the result does not depend on the plan.

constexpr uint32_t kNaWindow = 1u << 16;
constexpr uint64_t kNaClaims = 1ull << 22;
constexpr uint64_t kNaTailWords = kNaWindow + 32; // keys, count, left; padded to 256 bytes
constexpr uint64_t kNaPendWords = kNaWindow / 8;  // one flag byte per window key
constexpr uint64_t kNaScratchWords = kNaClaims + kNaTailWords + kNaPendWords;
static_assert(kNaWindow <= (1u << 24) - 1, "ages must fit below the step tag");

} // namespace

// 34,144,512 bytes per device, held from the library's first use of the
// device until the process ends: claim table | window tail keys, count, left
// | pending flags.
static __device__ __align__(256) uint64_t scratch[kNaScratchWords];

namespace {

constexpr int kNaMaxDevices = 64;

struct NoAllocDevice {
    uint64_t *ptr = nullptr; // scratch's device address on this device
    uint64_t tag = 0;        // last step tag written into its claim table
};

std::mutex g_na_mutex;
NoAllocDevice g_na[kNaMaxDevices];

template <int C>
hipError_t launch_det_noalloc_c(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    hipError_t e = prepare_ordered_c<C>(f);
    if (e != hipSuccess || n < kWideMinKeys)
        return e != hipSuccess ? e : enqueue_ordered_c<C>(f, keys, n, nullptr, s);
    if (f.device < 0 || f.device >= kNaMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_na_mutex);
    NoAllocDevice &d = g_na[f.device];
    if (d.ptr == nullptr) {
        // once per device, with the device current (the caller's guard made it
        // so): the array's address on this device, and a claim table cleared
        // below every tag, by a fill kernel on the caller's stream
        uint64_t *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        e = launch_fill_zero(ptr, kNaClaims, s);
        if (e != hipSuccess)
            return e;
        d.ptr = ptr;
    }
    const WidePlan plan{kNaWindow, kNaClaims, f.M >= (1ull << 24) ? 4 : 8};
    const WideScratch ws{d.ptr, reinterpret_cast<uint8_t *>(d.ptr + kNaClaims + kNaTailWords), d.ptr + kNaClaims,
                         &d.tag};
    return run_wide_c<C>(f, keys, n, plan, ws, s);
}

} // namespace

hipError_t launch_insert_det_noalloc(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    switch (f.c) {
    case 1:
        return launch_det_noalloc_c<1>(f, keys, n, s);
    case 2:
        return launch_det_noalloc_c<2>(f, keys, n, s);
    case 3:
        return launch_det_noalloc_c<3>(f, keys, n, s);
    case 4:
        return launch_det_noalloc_c<4>(f, keys, n, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_insert_det(bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s)
{
    switch (f.c) {
    case 1:
        return launch_det_c<1>(f, keys, n, s);
    case 2:
        return launch_det_c<2>(f, keys, n, s);
    case 3:
        return launch_det_c<3>(f, keys, n, s);
    case 4:
        return launch_det_c<4>(f, keys, n, s);
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace bbfc
