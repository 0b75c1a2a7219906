// Roofline probes: the memory access patterns of the filter kernels without
// the filter arithmetic. They measure what the device sustains for random
// 64-byte line reads and random 64-bit atomic ORs, eight lanes per line as
// in the insert and query kernels, and a plain streaming copy whose byte
// count calibrates the hardware traffic counters.
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "bbfc_internal.hpp"

namespace bbfc {

namespace {

constexpr int kProbeWG = 256;
constexpr int kProbeWave = 64;

// Counter-based line index (SplitMix64 finaliser of seed + i).
__device__ inline uint64_t probe_line(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Each wavefront handles 64 / LPL * 8 accesses per iteration: LPL lanes read
// one line of 8 * LPL bytes (lane w reads word w), eight rounds in flight.
template <int LPL>
__global__ __launch_bounds__(kProbeWG) void probe_gather_kernel(const uint64_t *__restrict__ buf, uint64_t line_mask,
                                                                uint64_t n_access, uint64_t seed,
                                                                uint64_t *__restrict__ sink)
{
    constexpr int kGroups = 64 / LPL;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = lane / LPL;
    const uint32_t w = lane % LPL;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint64_t acc = 0;
    for (uint64_t base = wave * kGroups * 8; base < n_access; base += n_waves * kGroups * 8) {
        uint64_t v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint64_t a = base + g * 8 + r;
            v[r] = 0;
            if (a < n_access)
                v[r] = buf[(probe_line(seed, a) & line_mask) * LPL + w];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
            acc += v[r];
    }
    // Stored only in the (practically impossible) case of a magic sum, so
    // the loads cannot be removed and nothing else is written.
    if (acc == 0x9E3779B97F4A7C15ull)
        sink[blockIdx.x & 0xFFFF] = acc;
}

__global__ __launch_bounds__(kProbeWG) void probe_atomic64_kernel(uint64_t *__restrict__ buf, uint64_t line_mask,
                                                                  uint64_t n_access, uint64_t seed)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = lane >> 3;
    const uint32_t w = lane & 7;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t base = wave * 64; base < n_access; base += n_waves * 64) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint64_t a = base + g * 8 + r;
            if (a < n_access) {
                const uint64_t h = probe_line(seed, a);
                __hip_atomic_fetch_or(&buf[(h & line_mask) * 8 + w], 1ull << ((h >> 58) ^ w), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ __launch_bounds__(kProbeWG) void probe_copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                              uint64_t n_vec)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vec; i += stride)
        dst[i] = src[i];
}

// The insert's memory pattern with a stand-in for its arithmetic: per key
// two random 64-byte lines are read (eight lanes per line, eight keys per
// lane group in flight). With MASK_BITS > 0 the key then has a mask of that
// many random bit positions (positions may repeat, as in the filter) and the
// group picks the line that gains fewer new bits, one choice for all eight
// lanes, and ORs the mask into it with 64-bit atomics, only on the words that
// gain a bit. So each key rewrites at most one line, as the insert does, and
// that write waits for both reads.
__device__ inline uint64_t probe_mask_word(uint64_t seed, uint64_t key, uint32_t w, int mask_bits)
{
    uint64_t m = 0;
    uint64_t h = 0;
    for (int i = 0; i < mask_bits; ++i) {
        if (i % 7 == 0)
            h = probe_line(seed ^ 0x5851F42D4C957F2Dull, key * 5 + (uint64_t)(i / 7));
        const uint32_t pos = (uint32_t)(h & 511);
        h >>= 9;
        m |= (pos >> 6) == w ? 1ull << (pos & 63) : 0ull;
    }
    return m;
}

template <bool ATOMIC>
__global__ __launch_bounds__(kProbeWG) void probe_insert_pattern_kernel(uint64_t *__restrict__ buf, uint64_t line_mask,
                                                                        uint64_t n_keys, int mask_bits, uint64_t seed,
                                                                        uint64_t *__restrict__ sink)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = lane >> 3;
    const uint32_t w = lane & 7;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint64_t acc = 0;
    for (uint64_t base = wave * 64; base < n_keys; base += n_waves * 64) {
        uint64_t v0[8], v1[8], l0[8], l1[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint64_t key = base + g * 8 + r;
            const uint64_t h = probe_line(seed, key);
            l0[r] = h & line_mask;
            l1[r] = ((h >> 32) ^ (h << 7)) & line_mask;
            v0[r] = v1[r] = 0;
            if (key < n_keys) {
                v0[r] = buf[l0[r] * 8 + w];
                v1[r] = buf[l1[r] * 8 + w];
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint64_t key = base + g * 8 + r;
            if constexpr (ATOMIC) {
                // every lane takes part in the shuffles; keys past the end
                // have an empty mask and write nothing
                const uint64_t m = key < n_keys ? probe_mask_word(seed, key, w, mask_bits) : 0;
                int d = __popcll(m & ~v0[r]) - __popcll(m & ~v1[r]);
                d += __shfl_xor(d, 1);
                d += __shfl_xor(d, 2);
                d += __shfl_xor(d, 4);
                const bool second = d > 0;
                const uint64_t old = second ? v1[r] : v0[r];
                if (m & ~old)
                    __hip_atomic_fetch_or(&buf[(second ? l1[r] : l0[r]) * 8 + w], m, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            } else if (key < n_keys) {
                acc += v0[r] + v1[r];
            }
        }
    }
    if (acc == 0x9E3779B97F4A7C15ull)
        sink[blockIdx.x & 0xFFFF] = acc;
}

// Two other schedules of the insert's pattern (same keys, lines and masks as
// probe_insert_pattern_kernel<true>):
//   PIPELINED  a wavefront decides all 64 keys of its unit first, then
//              issues their atomics (every lane, an OR of 0 where its word
//              gains nothing) and right after them the next unit's line
//              reads, so no wait for reads ever covers the atomics;
//   BLIND      the line is chosen from the key alone (one hash bit), not
//              from the words read: the atomics no longer depend on the
//              reads and issue together with them. The words read are still
//              consumed (summed after the atomics are issued), so that the
//              loads are not dropped as dead code. This is not an insert
//              (the choice ignores the blocks); it shows what the same
//              traffic costs without the read-to-write dependency.
template <int MODE>
__global__ __launch_bounds__(kProbeWG) void probe_insert_schedule_kernel(uint64_t *__restrict__ buf,
                                                                          uint64_t line_mask, uint64_t n_keys,
                                                                          int mask_bits, uint64_t seed,
                                                                          uint64_t *__restrict__ sink)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = lane >> 3;
    const uint32_t w = lane & 7;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint64_t base = wave * 64;
    if (base >= n_keys)
        return;
    uint64_t v0[8], v1[8], l0[8], l1[8];
    auto read_unit = [&](uint64_t b) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint64_t h = probe_line(seed, b + g * 8 + r);
            l0[r] = h & line_mask;
            l1[r] = ((h >> 32) ^ (h << 7)) & line_mask;
            v0[r] = buf[l0[r] * 8 + w]; // lines are masked into the buffer, also past n_keys
            v1[r] = buf[l1[r] * 8 + w];
        }
    };
    uint64_t acc = 0; // BLIND: the words read feed only this, so the loads stay
    read_unit(base);
    for (;;) {
        uint64_t cl[8], cm[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint64_t key = base + g * 8 + r;
            const uint64_t m = key < n_keys ? probe_mask_word(seed, key, w, mask_bits) : 0;
            bool second;
            if constexpr (MODE == 1) {
                int d = __popcll(m & ~v0[r]) - __popcll(m & ~v1[r]);
                d += __shfl_xor(d, 1);
                d += __shfl_xor(d, 2);
                d += __shfl_xor(d, 4);
                second = d > 0;
                const uint64_t old = second ? v1[r] : v0[r];
                cm[r] = (m & ~old) ? m : 0ull;
            } else {
                second = (probe_line(seed ^ 0x632BE59BD9B4E019ull, key) >> 63) != 0;
                cm[r] = m;
            }
            cl[r] = second ? l1[r] : l0[r];
        }
        const uint64_t next = base + n_waves * 64;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            __hip_atomic_fetch_or(&buf[cl[r] * 8 + w], cm[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (MODE == 2) {
            // consumed after the atomics are issued: they do not wait for these reads
#pragma unroll
            for (int r = 0; r < 8; ++r)
                acc += v0[r] ^ v1[r];
        }
        if (next >= n_keys)
            break;
        base = next;
        read_unit(base);
    }
    if (acc == 0x9E3779B97F4A7C15ull)
        sink[blockIdx.x & 0xFFFF] = acc;
}

// 64-byte requests: a wavefront takes 8 consecutive 128-byte lines per
// unit; group g (lanes 8g..8g+7) moves the low 64-byte half of line g, then,
// in a second instruction, its high half.
__global__ __launch_bounds__(kProbeWG) void probe_copy64_kernel(const uint64_t *__restrict__ src,
                                                                uint64_t *__restrict__ dst, uint64_t n_units)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t g = lane >> 3;
    const uint64_t w = lane & 7;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t u = wave; u < n_units; u += n_waves) {
        const uint64_t line = (u * 8 + g) * 16;
        dst[line + w] = src[line + w];
        dst[line + 8 + w] = src[line + 8 + w];
    }
}

uint32_t probe_grid(const void *kernel)
{
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kProbeWG, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (cus < 1)
        cus = 1;
    return (uint32_t)(per_cu * cus);
}

} // namespace

// One wavefront per workgroup times `iters` dependent steps of one kind of
// memory round trip with the device's constant-rate clock and writes the
// mean nanoseconds per step to out[blockIdx.x]. Lanes 8g..8g+7 share one
// line, as in the filter kernels. kind 0: a random line read whose address
// depends on the previous read; 1: a random 64-bit atomic OR and the wait
// for it; 2: a random line read, then an atomic OR into the line just read,
// and the wait for both; 3: a coalesced 512-byte load of fresh words, its
// address depending on the previous load, and the wait for it.
__global__ __launch_bounds__(kProbeWave) void probe_latency_kernel(uint64_t *__restrict__ buf, uint64_t line_mask,
                                                               int kind, uint32_t iters, double ns_per_tick,
                                                               double *__restrict__ out)
{
    const uint32_t lane = threadIdx.x;
    const uint32_t w = lane % 8;
    const uint64_t word_mask = line_mask * 8 + 7;
    uint64_t x = probe_line(0x5851F42D4C957F2Dull * (blockIdx.x + 1), lane / 8);
    uint64_t acc = 0;
    const uint64_t t0 = wall_clock64();
    for (uint32_t i = 0; i < iters; ++i) {
        if (kind == 0) {
            acc += buf[((x ^ acc) & line_mask) * 8 + w] + 1;
        } else if (kind == 1) {
            __hip_atomic_fetch_or(buf + (x & line_mask) * 8 + w, 1ull << (i & 63), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
        } else if (kind == 2) {
            uint64_t *word = buf + ((x ^ (acc & 1)) & line_mask) * 8 + w;
            const uint64_t v = *word;
            acc += v;
            __hip_atomic_fetch_or(word, (1ull << (i & 63)) | (v & 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
        } else {
            const uint64_t idx = ((uint64_t)i * gridDim.x + blockIdx.x) * kProbeWave + lane;
            acc += buf[(idx + (acc & 1)) & word_mask];
        }
        x = probe_line(x, i);
    }
    const uint64_t t1 = wall_clock64();
    // acc keeps the loads; the term it adds is below a double's resolution here
    const double keep = acc == 0x9E3779B97F4A7C15ull ? 1e-300 : 0.0;
    if (lane == 0)
        out[blockIdx.x] = (double)(t1 - t0) * ns_per_tick / iters + keep;
}

hipError_t launch_probe_gather(const uint64_t *buf, uint64_t n_lines64, uint32_t access_bytes, uint64_t n_access,
                               uint64_t seed, uint64_t *sink, hipStream_t s)
{
    const void *k = access_bytes == 128 ? (const void *)probe_gather_kernel<16> : (const void *)probe_gather_kernel<8>;
    uint32_t grid = probe_grid(k);
    const uint64_t need = (n_access + 255) / 256;
    if (need < grid)
        grid = (uint32_t)(need ? need : 1);
    const uint64_t lines = access_bytes == 128 ? n_lines64 / 2 : n_lines64;
    if (access_bytes == 128)
        hipLaunchKernelGGL(probe_gather_kernel<16>, dim3(grid), dim3(kProbeWG), 0, s, buf, lines - 1, n_access, seed,
                           sink);
    else
        hipLaunchKernelGGL(probe_gather_kernel<8>, dim3(grid), dim3(kProbeWG), 0, s, buf, lines - 1, n_access, seed,
                           sink);
    return hipGetLastError();
}

hipError_t launch_probe_atomic64(uint64_t *buf, uint64_t n_lines, uint64_t n_access, uint64_t seed, hipStream_t s)
{
    uint32_t grid = probe_grid((const void *)probe_atomic64_kernel);
    const uint64_t need = (n_access + 255) / 256;
    if (need < grid)
        grid = (uint32_t)(need ? need : 1);
    hipLaunchKernelGGL(probe_atomic64_kernel, dim3(grid), dim3(kProbeWG), 0, s, buf, n_lines - 1, n_access, seed);
    return hipGetLastError();
}

hipError_t launch_probe_insert_pattern(uint64_t *buf, uint64_t n_lines, uint64_t n_keys, int mask_bits, uint64_t seed,
                                       uint64_t *sink, hipStream_t s)
{
    const bool atomic = mask_bits > 0;
    const void *k = atomic ? (const void *)probe_insert_pattern_kernel<true>
                           : (const void *)probe_insert_pattern_kernel<false>;
    uint32_t grid = probe_grid(k);
    const uint64_t need = (n_keys + 255) / 256;
    if (need < grid)
        grid = (uint32_t)(need ? need : 1);
    if (atomic)
        hipLaunchKernelGGL(probe_insert_pattern_kernel<true>, dim3(grid), dim3(kProbeWG), 0, s, buf, n_lines - 1,
                           n_keys, mask_bits, seed, sink);
    else
        hipLaunchKernelGGL(probe_insert_pattern_kernel<false>, dim3(grid), dim3(kProbeWG), 0, s, buf, n_lines - 1,
                           n_keys, 0, seed, sink);
    return hipGetLastError();
}

hipError_t launch_probe_insert_schedule(uint64_t *buf, uint64_t n_lines, uint64_t n_keys, int mask_bits,
                                        int schedule, uint64_t seed, uint64_t *sink, hipStream_t s)
{
    if (schedule == 0)
        return launch_probe_insert_pattern(buf, n_lines, n_keys, mask_bits, seed, sink, s);
    const void *k = schedule == 1 ? (const void *)probe_insert_schedule_kernel<1>
                                  : (const void *)probe_insert_schedule_kernel<2>;
    uint32_t grid = probe_grid(k);
    const uint64_t need = (n_keys + 255) / 256;
    if (need < grid)
        grid = (uint32_t)(need ? need : 1);
    if (schedule == 1)
        hipLaunchKernelGGL(probe_insert_schedule_kernel<1>, dim3(grid), dim3(kProbeWG), 0, s, buf, n_lines - 1, n_keys,
                           mask_bits, seed, sink);
    else
        hipLaunchKernelGGL(probe_insert_schedule_kernel<2>, dim3(grid), dim3(kProbeWG), 0, s, buf, n_lines - 1, n_keys,
                           mask_bits, seed, sink);
    return hipGetLastError();
}

hipError_t launch_probe_latency(uint64_t *buf, uint64_t n_lines, int kind, uint32_t iters, uint32_t waves,
                                double *out, hipStream_t s)
{
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess)
        return e;
    if (khz <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(probe_latency_kernel, dim3(waves), dim3(kProbeWave), 0, s, buf, n_lines - 1, kind, iters,
                       1e6 / (double)khz, out);
    return hipGetLastError();
}

hipError_t launch_probe_copy(const uint64_t *src, uint64_t *dst, uint64_t n_words, uint32_t request_bytes,
                             hipStream_t s)
{
    if (request_bytes == 64) {
        const uint64_t n_units = n_words / 128; // 8 lines of 16 words; the caller checked divisibility
        const uint32_t grid = probe_grid((const void *)probe_copy64_kernel) * 2;
        hipLaunchKernelGGL(probe_copy64_kernel, dim3(grid), dim3(kProbeWG), 0, s, src, dst, n_units);
        return hipGetLastError();
    }
    const uint64_t n_vec = n_words / 2; // whole 16-byte vectors; an odd last word is not copied
    uint32_t grid = probe_grid((const void *)probe_copy_kernel) * 2;
    hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(kProbeWG), 0, s, reinterpret_cast<const uint4 *>(src),
                       reinterpret_cast<uint4 *>(dst), n_vec);
    return hipGetLastError();
}

} // namespace bbfc
