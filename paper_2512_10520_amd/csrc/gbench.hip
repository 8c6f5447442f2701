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

// Issue-rate microbenchmark: 8 chains per thread updated in place, each
// update one VALU instruction of the chosen kind (the loop body is 8 such
// instructions and a scalar loop counter; checked in the gfx950 assembly):
//   0 v_fmac_f32      a_i += a_(i+1) * h
//   1 v_add_f32       a_i += a_(i+1)
//   2 v_lshl_add_u32  a_i = (a_i << 1) + a_(i+1)
//   3 v_fmac_f64      a_i += a_(i+1) * h
//   4 v_mad_u64_u32   a_i += lo(a_(i+1)) * K
// so a full grid measures how many wave-level instructions of that kind a
// SIMD completes per cycle.
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_valu(int iters, uint32_t seed, unsigned int *sink) {
    T a[8];
    const uint32_t t = seed ^ (blockIdx.x * blockDim.x + threadIdx.x);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = (T)(t + 977u * (uint32_t)i);
    const T h = (T)0.5;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {      // in place: chain 7 reads chain 0's new value
            const T nxt = a[(i + 1) & 7];
            if constexpr (KIND == 0 || KIND == 3) a[i] = fma(nxt, h, a[i]);
            else if constexpr (KIND == 1) a[i] = a[i] + nxt;
            else if constexpr (KIND == 2) a[i] = (a[i] << 1) + nxt;
            else a[i] = (uint64_t)(uint32_t)nxt * 0xD2511F53ull + a[i];
        }
    }
    T acc = a[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) acc = acc + a[i];
    if (acc == (T)0x12345) atomicAdd(sink, 1u);     // keeps the chains alive
}

}  // namespace

extern "C" int mtb_valu(int kind, int iters, int blocks, uint32_t seed, unsigned int *sink,
                        void *stream) {
    if (!sink || iters < 1 || blocks < 1 || kind < 0 || kind > 4) return -1;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (kind) {
    case 0: hipLaunchKernelGGL((k_valu<float, 0>), dim3(blocks), dim3(256), 0, st, iters, seed, sink); break;
    case 1: hipLaunchKernelGGL((k_valu<float, 1>), dim3(blocks), dim3(256), 0, st, iters, seed, sink); break;
    case 2: hipLaunchKernelGGL((k_valu<uint32_t, 2>), dim3(blocks), dim3(256), 0, st, iters, seed, sink); break;
    case 3: hipLaunchKernelGGL((k_valu<double, 3>), dim3(blocks), dim3(256), 0, st, iters, seed, sink); break;
    default: hipLaunchKernelGGL((k_valu<uint64_t, 4>), dim3(blocks), dim3(256), 0, st, iters, seed, sink); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

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
