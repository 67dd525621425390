// Read bandwidth of the LDS, for pricing LDS-bound kernels against what the
// hardware delivers rather than a nominal figure.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace asynet {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 8;

// Every wave reads consecutive elements (conflict-free, one element per lane),
// kProbeUnroll reads per pass, the same addresses each pass.  The empty asm
// with a memory clobber keeps the compiler from reusing the values of one pass
// in the next, so each pass issues its LDS reads again.
template <typename T>
__global__ void __launch_bounds__(kProbeThreads) lds_read_probe_kernel(int passes, uint32_t *sink)
{
    constexpr int kElems = kProbeThreads * kProbeUnroll;
    __shared__ T buf[kElems];
    constexpr int kWords = sizeof(T) / 4;
    for (int i = threadIdx.x; i < kElems; i += kProbeThreads) {
        uint32_t w[kWords];
#pragma unroll
        for (int c = 0; c < kWords; ++c)
            w[c] = (uint32_t)(i * 2654435761u + c);
        __builtin_memcpy(&buf[i], w, sizeof(T));
    }
    __syncthreads();
    uint32_t acc = 0;
    for (int p = 0; p < passes; ++p) {
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const T v = buf[u * kProbeThreads + threadIdx.x];
            uint32_t w[kWords];
            __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
            for (int c = 0; c < kWords; ++c)
                acc ^= w[c];
        }
        asm volatile("" ::: "memory");
    }
    sink[blockIdx.x * kProbeThreads + threadIdx.x] = acc;
}

}  // namespace asynet
