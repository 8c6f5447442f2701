// Gather microbenchmark: the rate of independent, uniformly random loads of
// 4 or 16 bytes from a buffer of a given size at full occupancy.  It sets the
// "gather" ceiling a table-driven step could reach if it were bound by its
// dependent table loads rather than by arithmetic.  Measurement only; not
// part of the transport library.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// One xorshift32 stream per thread; each load's address comes from its own
// stream value, so the loads of a thread are independent of the data read.
template <int WIDTH>
__global__ void __launch_bounds__(256) k_gather(const char *buf, uint32_t n_items, int loads,
                                                uint32_t seed, unsigned int *sink) {
    uint32_t x = seed ^ (blockIdx.x * blockDim.x + threadIdx.x) * 0x9E3779B9u;
    x = x ? x : 1u;
    uint32_t acc = 0;
    for (int i = 0; i < loads; ++i) {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        const uint32_t idx = __umulhi(x, n_items);
        if (WIDTH == 16) {
            const uint4 v = reinterpret_cast<const uint4 *>(buf)[idx];
            acc += v.x ^ v.y ^ v.z ^ v.w;
        } else {
            acc += reinterpret_cast<const uint32_t *>(buf)[idx];
        }
    }
    if (acc == 0x12345678u) atomicAdd(sink, 1u);     // keeps the loads alive
}

}  // namespace

extern "C" int mtb_gather(const void *buf, uint64_t bytes, int width, int loads, int blocks,
                          uint32_t seed, unsigned int *sink, void *stream) {
    if (!buf || !sink || (width != 4 && width != 16) || loads < 1 || blocks < 1) return -1;
    const uint64_t n = bytes / (uint64_t)width;
    if (n < 1 || n > 0xFFFFFFFFull) return -1;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (width == 16)
        hipLaunchKernelGGL(k_gather<16>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const char *>(buf), (uint32_t)n, loads, seed, sink);
    else
        hipLaunchKernelGGL(k_gather<4>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const char *>(buf), (uint32_t)n, loads, seed, sink);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}
