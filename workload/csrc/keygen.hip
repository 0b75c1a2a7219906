// Device-side generator of the seeded synthetic keys: the same counter-based
// SplitMix64 stream as the numpy generator in this module,
//   key(seed, i) = mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)  (mod 2^64),
// so that billions of keys can be made directly in device memory. No filter
// arithmetic lives here.
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace {

__global__ void splitmix_keys_kernel(uint64_t seed, uint64_t start, uint64_t n, uint64_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t z = seed + (start + i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        out[i] = z ^ (z >> 31);
    }
}

} // namespace

extern "C" int wl_splitmix64_keys(uint64_t seed, uint64_t start, uint64_t n, uint64_t *d_out, hipStream_t stream)
{
    if (n == 0)
        return 0;
    if (d_out == nullptr)
        return -1;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384)
        blocks = 16384;
    hipLaunchKernelGGL(splitmix_keys_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, seed, start, n, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Reads of read_len bases sampled from a packed genome (32 bases per word,
// base i in bits 63-2(i%32) .. 62-2(i%32) of word i/32), concatenated and
// packed the same way. Read r starts at mix(seed, r) mod (genome - read_len
// + 1) and is the reverse complement when bit 0 of mix(seed ^ S1, r) is set;
// base p of the output is replaced by one of the three other bases when
// mix(seed ^ S2, p) < err_threshold (probability err_threshold / 2^64), the
// replacement chosen by mix(seed ^ S3, p) mod 3. One thread writes one word.
namespace {

__device__ inline uint64_t wl_mix(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr uint64_t kStrandSalt = 0xA5A5A5A5A5A5A5A5ull;
constexpr uint64_t kErrSalt = 0x5A5A5A5A5A5A5A5Aull;
constexpr uint64_t kSubSalt = 0x3C3C3C3C3C3C3C3Cull;

__global__ void reads_kernel(const uint64_t *__restrict__ genome, uint64_t n_genome, uint64_t n_reads,
                             uint64_t read_len, uint64_t err_threshold, uint64_t seed, uint64_t *__restrict__ out,
                             uint64_t n_words)
{
    const uint64_t total = n_reads * read_len;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_words; w += stride) {
        uint64_t p = w * 32;
        uint64_t r = p / read_len;
        uint64_t j = p - r * read_len;
        uint64_t start = 0, strand = 0;
        uint64_t cur = ~0ull;
        uint64_t word = 0;
        for (int b = 0; b < 32; ++b, ++p, ++j) {
            if (j == read_len) {
                j = 0;
                ++r;
            }
            uint64_t base = 0;
            if (p < total) {
                if (r != cur) {
                    start = wl_mix(seed, r) % (n_genome - read_len + 1);
                    strand = wl_mix(seed ^ kStrandSalt, r) & 1;
                    cur = r;
                }
                const uint64_t g = start + (strand ? read_len - 1 - j : j);
                base = (genome[g >> 5] >> (62 - 2 * (g & 31))) & 3;
                if (strand)
                    base = 3 - base;
                if (wl_mix(seed ^ kErrSalt, p) < err_threshold)
                    base = (base + 1 + wl_mix(seed ^ kSubSalt, p) % 3) & 3;
            }
            word |= base << (62 - 2 * b);
        }
        out[w] = word;
    }
}

} // namespace

extern "C" int wl_reads(const uint64_t *d_genome, uint64_t n_genome, uint64_t n_reads, uint64_t read_len,
                        uint64_t err_threshold, uint64_t seed, uint64_t *d_out, hipStream_t stream)
{
    if (n_reads == 0 || read_len == 0)
        return 0;
    if (d_genome == nullptr || d_out == nullptr || n_genome < read_len)
        return -1;
    const uint64_t n_words = (n_reads * read_len + 31) / 32;
    uint64_t blocks = (n_words + 255) / 256;
    if (blocks > 16384)
        blocks = 16384;
    hipLaunchKernelGGL(reads_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, d_genome, n_genome, n_reads,
                       read_len, err_threshold, seed, d_out, n_words);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Planted repeats: bases of the output genome equal the input genome, except
// inside segments [dst_s, dst_s + len_s) (sorted by dst, non-overlapping),
// which copy the input from src_s on; base p of a copy is replaced by one of
// the three other bases when mix(seed ^ S4, p) < div_threshold, the
// replacement chosen by mix(seed ^ S5, p) mod 3. One thread writes one word.
namespace {

constexpr uint64_t kPlantErrSalt = 0x6B6B6B6B6B6B6B6Bull;
constexpr uint64_t kPlantSubSalt = 0x1E1E1E1E1E1E1E1Eull;

__device__ inline uint64_t base_at(const uint64_t *__restrict__ g, uint64_t i)
{
    return (g[i >> 5] >> (62 - 2 * (i & 31))) & 3;
}

__global__ void plant_kernel(const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint64_t n_bases,
                             const uint64_t *__restrict__ dst, const uint64_t *__restrict__ len,
                             const uint64_t *__restrict__ src, uint64_t n_seg, uint64_t div_threshold, uint64_t seed)
{
    const uint64_t n_words = (n_bases + 31) / 32;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_words; w += stride) {
        const uint64_t p0 = w * 32;
        // last segment starting at or before p0 (n_seg if none)
        uint64_t lo = 0, hi = n_seg;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            if (dst[mid] <= p0)
                lo = mid + 1;
            else
                hi = mid;
        }
        uint64_t s = lo == 0 ? n_seg : lo - 1;
        uint64_t word = in[w];
        for (int b = 0; b < 32; ++b) {
            const uint64_t p = p0 + b;
            if (p >= n_bases)
                break;
            const uint64_t nxt = s == n_seg ? 0 : s + 1;
            if (nxt < n_seg && dst[nxt] <= p)
                s = nxt;
            if (s < n_seg && p >= dst[s] && p < dst[s] + len[s]) {
                uint64_t base = base_at(in, src[s] + (p - dst[s]));
                if (wl_mix(seed ^ kPlantErrSalt, p) < div_threshold)
                    base = (base + 1 + wl_mix(seed ^ kPlantSubSalt, p) % 3) & 3;
                const int sh = 62 - 2 * b;
                word = (word & ~(3ull << sh)) | (base << sh);
            }
        }
        out[w] = word;
    }
}

} // namespace

extern "C" int wl_plant(const uint64_t *d_in, uint64_t *d_out, uint64_t n_bases, const uint64_t *d_dst,
                        const uint64_t *d_len, const uint64_t *d_src, uint64_t n_seg, uint64_t div_threshold,
                        uint64_t seed, hipStream_t stream)
{
    if (n_bases == 0)
        return 0;
    if (d_in == nullptr || d_out == nullptr || (n_seg > 0 && (d_dst == nullptr || d_len == nullptr || d_src == nullptr)))
        return -1;
    const uint64_t n_words = (n_bases + 31) / 32;
    uint64_t blocks = (n_words + 255) / 256;
    if (blocks > 16384)
        blocks = 16384;
    hipLaunchKernelGGL(plant_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, d_in, d_out, n_bases, d_dst, d_len,
                       d_src, n_seg, div_threshold, seed);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
