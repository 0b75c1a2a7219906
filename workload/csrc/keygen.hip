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
