// Random-access reference kernel (see tw_probe.h).  Each thread draws its
// buffer positions from splitmix64 of (thread, step), so no index array is
// read; the loaded words are folded into a value that is stored only if it
// matches a constant, which keeps the loads alive at no traffic.
#include "tw_probe.h"

namespace twk {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int kMode>
__global__ __launch_bounds__(kProbeBlock) void probe_rate_kernel(uint4 *buf, uint64_t n16, uint64_t per_thread,
                                                                 uint32_t *sink)
{
    const uint64_t tid = (uint64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    uint32_t acc = 0;
    if (kMode == 2) {
        for (uint64_t i = 0; i + 8 <= per_thread; i += 8) {
            uint4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = buf[__umul64hi(mix64(tid * per_thread + i + u), n16)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                acc ^= v[u].x ^ v[u].w;
        }
    } else {
#pragma unroll 1
        for (uint64_t i = 0; i < per_thread; ++i) {
            const uint64_t h = mix64(tid * per_thread + i);
            const uint64_t b = __umul64hi(h, n16);
            if (kMode == 0) {
                const uint4 v = buf[b];
                acc ^= v.x ^ v.w;
            } else if (kMode == 3) {
                using Vec = unsigned __attribute__((ext_vector_type(4)));
                const Vec v = __builtin_nontemporal_load((const Vec *)&buf[b]);
                acc ^= v.x ^ v.w;
            } else if (kMode == 4) {
                const uint64_t v = *(const uint64_t *)&buf[b];
                acc ^= (uint32_t)v ^ (uint32_t)(v >> 32);
            } else if (kMode == 5) {
                const uint64_t v = __hip_atomic_load((const uint64_t *)&buf[b], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_SYSTEM);
                acc ^= (uint32_t)v ^ (uint32_t)(v >> 32);
            } else {
                unsigned long long *p = (unsigned long long *)&buf[b];
                acc ^= (uint32_t)atomicCAS(p, ~0ull, (unsigned long long)(h | 1ull));
            }
        }
    }
    if (acc == 0x9E3779B9u)
        sink[0] = acc;
}

}  // namespace

hipError_t launch_probe_rate(void *buf, uint64_t bytes, uint64_t per_thread, int mode, unsigned blocks,
                             uint32_t *sink, hipStream_t s)
{
    const uint64_t n16 = bytes / 16;
    if (n16 == 0 || per_thread == 0)
        return hipSuccess;
    if (mode == 0)
        hipLaunchKernelGGL(probe_rate_kernel<0>, dim3(blocks), dim3(kProbeBlock), 0, s, (uint4 *)buf, n16,
                           per_thread, sink);
    else if (mode == 1)
        hipLaunchKernelGGL(probe_rate_kernel<1>, dim3(blocks), dim3(kProbeBlock), 0, s, (uint4 *)buf, n16,
                           per_thread, sink);
    else if (mode == 2)
        hipLaunchKernelGGL(probe_rate_kernel<2>, dim3(blocks), dim3(kProbeBlock), 0, s, (uint4 *)buf, n16,
                           per_thread, sink);
    else if (mode == 3)
        hipLaunchKernelGGL(probe_rate_kernel<3>, dim3(blocks), dim3(kProbeBlock), 0, s, (uint4 *)buf, n16,
                           per_thread, sink);
    else if (mode == 4)
        hipLaunchKernelGGL(probe_rate_kernel<4>, dim3(blocks), dim3(kProbeBlock), 0, s, (uint4 *)buf, n16,
                           per_thread, sink);
    else
        hipLaunchKernelGGL(probe_rate_kernel<5>, dim3(blocks), dim3(kProbeBlock), 0, s, (uint4 *)buf, n16,
                           per_thread, sink);
    return hipGetLastError();
}

}  // namespace twk
